// Serving loop: requests arrive at any time, are admitted by device-memory
// budget and slots, stay resident on the device, and advance in rounds. Each
// round runs one quantum of every resident request in one batched persistent
// launch (stencil_batch_submit), so requests that arrive while others run are
// batched with them from a following round on (continuous batching). A
// quantum is a few passes of the request's temporal depth; running T steps as
// several quanta is the same arithmetic as one run, so results do not depend
// on the mix. By default the next round is composed when the running one
// has ended; with two rounds in flight it is composed and enqueued shortly
// before the running one is expected to end, so the device does not wait on
// the host between rounds (measured on MI355X: lower latency under moderate
// load, but smaller rounds and lower capacity under saturation).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "plan.hpp"
#include "server_admission.hpp"

using namespace stencil_impl;

namespace {

using Clock = std::chrono::steady_clock;

enum class RState { kQueued, kResident, kDone, kFailed };

// Pinned host blocks in power-of-two size classes, reused across requests:
// copies between pinned memory and the device go by DMA, while pageable
// copies go through staging kernels that compete with the stencil kernels.
class PinnedPool {
 public:
  ~PinnedPool() {
    for (auto& kv : free_) (void)hipHostFree(kv.second);
  }
  static size_t size_class(size_t bytes) {
    size_t c = (size_t)1 << 20;
    while (c < bytes) c <<= 1;
    return c;
  }
  void* get(size_t bytes, size_t* cls) {
    *cls = size_class(bytes);
    {
      std::lock_guard<std::mutex> lock(mu_);
      auto it = free_.find(*cls);
      if (it != free_.end()) {
        void* p = it->second;
        free_.erase(it);
        return p;
      }
    }
    void* p = nullptr;
    if (hipHostMalloc(&p, *cls, hipHostMallocDefault) != hipSuccess) return nullptr;
    return p;
  }
  void put(void* p, size_t cls) {
    if (!p) return;
    std::lock_guard<std::mutex> lock(mu_);
    free_.emplace(cls, p);
  }

 private:
  std::mutex mu_;
  std::multimap<size_t, void*> free_;
};

// Host copy of a request's grid into or out of pinned staging. One thread
// copies at about 7 GB/s, so a 13 MB grid takes about 2 ms of the caller's
// submit or wait: under load that, not the device, bounded the requests a
// client could put through. Large copies are split over a few threads.
void staging_copy(void* dst, const void* src, size_t bytes) {
  constexpr size_t kSplit = (size_t)4 << 20;  // below this one thread copies
  constexpr int kThreads = 4;
  if (bytes < kSplit) {
    std::memcpy(dst, src, bytes);
    return;
  }
  const size_t part = (bytes / kThreads + 4095) / 4096 * 4096;
  std::thread helpers[kThreads - 1];
  int started = 0;
  for (int k = 1; k < kThreads; ++k) {
    const size_t off = (size_t)k * part;
    if (off >= bytes) break;
    const size_t len = std::min(part, bytes - off);
    try {
      helpers[started] = std::thread(
          [=] { std::memcpy((char*)dst + off, (const char*)src + off, len); });
      ++started;
    } catch (...) {  // no thread: copy this part here
      std::memcpy((char*)dst + off, (const char*)src + off, len);
    }
  }
  std::memcpy(dst, src, std::min(part, bytes));
  for (int k = 0; k < started; ++k) helpers[k].join();
}

struct Request {
  uint64_t ticket = 0;
  // the batched plan, made once at submit; each round runs a copy
  // rescheduled for its steps
  std::unique_ptr<stencil_plan_s> plan;
  void* host_in = nullptr;  // pinned copy of the input (released once uploaded)
  size_t host_cls = 0;
  size_t bytes = 0;  // one padded grid
  size_t need = 0;   // device bytes held while resident
  int64_t remaining = 0;    // steps not yet completed
  int64_t unscheduled = 0;  // steps not yet in an enqueued round
  bool scheduled = false;   // in an enqueued round at least once (T = 0 runs once)
  int64_t depth = 1;    // steps per pass of the batched plan
  int64_t cells = 1;
  char* dev = nullptr;  // two padded grids
  int cur = 0;          // which half holds the state after the completed rounds
  int cur_next = 0;     // which half the next enqueued round reads
  RState state = RState::kQueued;
  bool collecting = false;
  stencil_status err = STENCIL_OK;
  Clock::time_point t_submit, t_done;
  double updates = 0;
  void* grid(int k) const { return dev + (size_t)k * ((bytes + 255) / 256 * 256); }
};

// A round in flight: its requests and their steps, the event recorded after
// its launches, and the pinned word that receives the compute stream's report
// word (watchdog expiries) just before that event, so that a round's outcome
// is known without waiting for the round enqueued after it.
struct Round {
  std::vector<Request*> reqs;
  std::vector<int64_t> steps;
  hipEvent_t done = nullptr;
  unsigned int* report = nullptr;
  double updates = 0;
  Clock::time_point t0;
  stencil_status st = STENCIL_OK;  // status of enqueueing it
};

constexpr int kMaxRoundsInFlight = 2;
// With two rounds in flight the next round is composed this long before the
// running one is expected to end (its cell-updates at the measured
// throughput): late enough that the arrivals admitted meanwhile join it,
// early enough to hide the host's work between rounds.
constexpr double kComposeLead_s = 2e-3;

// An admission's upload on the copy stream, marked by an event; the pinned
// input block goes back to the pool as soon as the event completes.
struct Upload {
  hipEvent_t done = nullptr;
  uint64_t ticket = 0;
};

}  // namespace

struct stencil_server_s {
  stencil_server_config cfg;
  hipStream_t compute = nullptr, copy = nullptr, collect = nullptr;
  // the server's own stream-ordered pool: request grids and round workspaces
  // come from it, and it keeps freed memory up to the budget instead of
  // returning it to the runtime at every synchronisation (the default pool's
  // behaviour), so admissions reuse memory rather than map new pages while
  // the scheduler holds the lock
  hipMemPool_t pool = nullptr;
  hipEvent_t inputs_ready = nullptr, copy_mark = nullptr;
  Round rounds[kMaxRoundsInFlight];
  std::deque<int> inflight;  // indices into rounds, oldest first
  std::deque<Upload> uploads;  // in copy-stream order
  Clock::time_point last_round_end;
  std::mutex mu;
  std::condition_variable cv_work;  // new submissions or stop
  std::condition_variable cv_done;  // a request finished
  Admission<Request> adm;  // queue, resident requests, budget and slots
  std::map<uint64_t, std::unique_ptr<Request>> all;
  uint64_t next_ticket = 1;
  double rate = 3.0e11;  // cell-updates per second, running estimate over rounds
  bool stop = false;
  bool pending_inputs = false;  // copies enqueued since the last round started
  std::thread worker;
  // statistics
  stencil_server_statistics st;
  std::vector<double> latencies;
  bool any_submit = false;
  Clock::time_point first_submit, last_done;
  std::mutex collect_mu;
  PinnedPool pinned;
};

namespace {

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

void finish_locked(stencil_server_s* srv, Request* r, RState s, stencil_status err) {
  r->state = s;
  r->err = err;
  r->t_done = Clock::now();
  if (s == RState::kDone) {
    const double lat = std::chrono::duration<double>(r->t_done - r->t_submit).count();
    srv->latencies.push_back(lat);
    srv->st.completed++;
    srv->st.cell_updates += r->updates;
    srv->last_done = r->t_done;
  } else {
    srv->st.failed++;
  }
}

// Admit queued requests in arrival order while a slot and the budget allow;
// their inputs are copied on the copy stream. Called with srv->mu held.
void admit_locked(stencil_server_s* srv) {
  srv->adm.admit([&](Request* r) {
    const size_t two = 2 * align256(r->bytes);
    hipError_t e = hipMallocFromPoolAsync((void**)&r->dev, two, srv->pool, srv->copy);
    if (e == hipSuccess)
      e = hipMemcpyAsync(r->dev, r->host_in, r->bytes, hipMemcpyHostToDevice, srv->copy);
    if (e == hipSuccess) {
      // without an event the block is released when the request's first
      // round completes instead
      Upload u;
      u.ticket = r->ticket;
      if (hipEventCreateWithFlags(&u.done, hipEventDisableTiming) == hipSuccess) {
        if (hipEventRecord(u.done, srv->copy) == hipSuccess) srv->uploads.push_back(u);
        else (void)hipEventDestroy(u.done);
      }
    }
    if (e != hipSuccess) {
      if (r->dev) (void)hipFreeAsync(r->dev, srv->copy);
      r->dev = nullptr;
      r->state = RState::kFailed;
      r->err = STENCIL_ERR_NOMEM;
      r->t_done = Clock::now();
      srv->st.failed++;
      srv->cv_done.notify_all();
      return false;
    }
    srv->st.admitted++;
    srv->pending_inputs = true;
    // (a T = 0 request also runs in a round: its job is a device copy on the
    // compute stream, ordered after the upload like every other job)
    r->state = RState::kResident;
    return true;
  });
  srv->st.hbm_in_use = srv->adm.in_use;
  srv->st.hbm_peak = srv->adm.peak;
  int active = 0;
  for (Request* r : srv->adm.resident) active += r->state == RState::kResident;
  srv->st.active = active;
  srv->st.max_active = std::max(srv->st.max_active, active);
  srv->st.queued = (int32_t)srv->adm.queue.size();
}

// Gives the pinned input blocks of completed uploads back to the pool (the
// copy stream runs them in order, so the first pending one ends the scan).
// Called with the lock held.
void reap_uploads_locked(stencil_server_s* srv) {
  while (!srv->uploads.empty()) {
    Upload& u = srv->uploads.front();
    const hipError_t q = hipEventQuery(u.done);
    if (q == hipErrorNotReady) break;
    auto it = srv->all.find(u.ticket);
    if (q == hipSuccess && it != srv->all.end() && it->second->host_in) {
      Request* r = it->second.get();
      srv->pinned.put(r->host_in, r->host_cls);
      r->host_in = nullptr;
    }
    (void)hipEventDestroy(u.done);
    srv->uploads.pop_front();
  }
}

// Whether a resident request still has steps to put into a round.
bool schedulable(const Request* r) {
  return r->state == RState::kResident && (r->unscheduled > 0 || !r->scheduled);
}

// Composes the next round from the resident requests and enqueues it on the
// compute stream into rounds[slot]. Called with the lock held; releases it
// while enqueueing. Returns false when no request has steps left to schedule.
bool enqueue_round(stencil_server_s* srv, std::unique_lock<std::mutex>& lock, int slot) {
  Round& R = srv->rounds[slot];
  R.reqs.clear();
  R.steps.clear();
  for (Request* r : srv->adm.resident)
    if (schedulable(r)) R.reqs.push_back(r);
  if (R.reqs.empty()) return false;
  // one quantum of every request: its fair share of the round's work, in
  // whole passes
  const size_t n = R.reqs.size();
  std::vector<const stencil_plan_s*> plans(n);
  std::vector<const void*> ins(n);
  std::vector<void*> outs(n);
  const double share = srv->cfg.round_target_s > 0 ? srv->cfg.round_target_s * srv->rate / (double)n : 0.0;
  R.updates = 0;
  for (size_t k = 0; k < n; ++k) {
    Request* r = R.reqs[k];
    int64_t q = (int64_t)(share / (double)r->cells) / r->depth * r->depth;
    q = std::max<int64_t>(q, (int64_t)srv->cfg.quantum_passes * r->depth);
    const int64_t steps = std::min(r->unscheduled, q);
    R.steps.push_back(steps);
    R.updates += (double)steps * (double)r->cells;
    plans[k] = r->plan.get();
    ins[k] = r->grid(r->cur_next);
    outs[k] = r->grid(1 - r->cur_next);
    // the request's state as the rounds enqueued so far leave it
    r->unscheduled -= steps;
    r->cur_next = 1 - r->cur_next;
    r->scheduled = true;
  }
  const bool wait_inputs = srv->pending_inputs;
  srv->pending_inputs = false;
  lock.unlock();
  R.t0 = Clock::now();
  stencil_status st = STENCIL_OK;
  if (wait_inputs) {
    // admissions copied since the last round: their inputs first
    if (hipEventRecord(srv->inputs_ready, srv->copy) != hipSuccess ||
        hipStreamWaitEvent(srv->compute, srv->inputs_ready, 0) != hipSuccess)
      st = hip_fail(hipErrorUnknown, "server input ordering");
  }
  if (st == STENCIL_OK) st = batch_submit_planned(plans, R.steps, ins, outs, srv->compute, srv->pool);
  if (st == STENCIL_OK) {
    unsigned int* word = stream_report_word(srv->compute);
    hipError_t e = word ? hipMemcpyAsync(R.report, word, sizeof(unsigned int), hipMemcpyDeviceToHost, srv->compute)
                        : hipErrorOutOfMemory;
    if (e == hipSuccess) e = hipEventRecord(R.done, srv->compute);
    if (e != hipSuccess) st = hip_fail(e, "server round event");
  }
  R.st = st;
  lock.lock();
  srv->inflight.push_back(slot);
  return true;
}

// Fails every request of every round in flight (after a failed enqueue or an
// expired device wait) once the compute stream is idle, and clears the
// stream's report word. Called with the lock held; releases it while waiting.
void fail_inflight(stencil_server_s* srv, std::unique_lock<std::mutex>& lock, stencil_status st) {
  lock.unlock();
  (void)hipStreamSynchronize(srv->compute);
  (void)stencil_sync(srv->compute);  // reads and clears the report word
  lock.lock();
  for (int slot : srv->inflight) {
    Round& R = srv->rounds[slot];
    srv->st.rounds++;
    for (Request* r : R.reqs) {
      if (r->host_in) {
        srv->pinned.put(r->host_in, r->host_cls);
        r->host_in = nullptr;
      }
      if (r->state == RState::kResident) finish_locked(srv, r, RState::kFailed, st);
    }
    R.reqs.clear();
  }
  srv->inflight.clear();
  srv->cv_done.notify_all();
}

// Retires the oldest round, which has completed: its requests advance, and
// those with no steps left are done. Called with the lock held.
void retire_round(stencil_server_s* srv) {
  const int slot = srv->inflight.front();
  srv->inflight.pop_front();
  Round& R = srv->rounds[slot];
  const Clock::time_point now = Clock::now();
  // busy time of this round: from its enqueue or the previous round's end,
  // whichever is later (the rounds overlap in the queue, not on the device)
  const Clock::time_point from = std::max(R.t0, srv->last_round_end);
  const double busy = std::chrono::duration<double>(now - from).count();
  srv->last_round_end = now;
  srv->st.rounds++;
  srv->st.busy_s += busy;
  if (busy > 0) {
    // throughput of this round, smoothed; small rounds under-fill the
    // device, so only rounds near the target duration update it upward
    const double r_now = R.updates / busy;
    if (srv->cfg.round_target_s <= 0 || busy >= 0.5 * srv->cfg.round_target_s || r_now < srv->rate)
      srv->rate = 0.7 * srv->rate + 0.3 * r_now;
  }
  for (size_t k = 0; k < R.reqs.size(); ++k) {
    Request* r = R.reqs[k];
    if (r->host_in) {  // its upload finished before its first round started
      srv->pinned.put(r->host_in, r->host_cls);
      r->host_in = nullptr;
    }
    r->cur = 1 - r->cur;
    r->remaining -= R.steps[k];
    if (r->remaining == 0 && r->unscheduled == 0) finish_locked(srv, r, RState::kDone, STENCIL_OK);
  }
  R.reqs.clear();
  srv->cv_done.notify_all();
}

// Whether the next round should be composed now: no round is in flight, or
// the oldest one is expected to end within the lead. Called with the lock held.
bool compose_now(const stencil_server_s* srv) {
  if (srv->inflight.empty()) return true;
  if ((int)srv->inflight.size() >= srv->cfg.rounds_in_flight) return false;
  const Round& R = srv->rounds[srv->inflight.front()];
  const Clock::time_point start = std::max(R.t0, srv->last_round_end);
  const double expected = R.updates / std::max(srv->rate, 1e9) - kComposeLead_s;
  return std::chrono::duration<double>(Clock::now() - start).count() >= expected;
}

void scheduler(stencil_server_s* srv) {
  (void)hipSetDevice(srv->cfg.device);
  std::unique_lock<std::mutex> lock(srv->mu);
  while (!srv->stop) {
    admit_locked(srv);
    reap_uploads_locked(srv);
    // the next round, enqueued behind the running one near its end
    if (compose_now(srv)) {
      int slot = 0;
      while (slot < kMaxRoundsInFlight &&
             std::find(srv->inflight.begin(), srv->inflight.end(), slot) != srv->inflight.end())
        ++slot;
      if (enqueue_round(srv, lock, slot)) {
        if (srv->rounds[slot].st != STENCIL_OK) fail_inflight(srv, lock, srv->rounds[slot].st);
        continue;
      }
    }
    if (srv->inflight.empty()) {
      // sleep until a queued request fits (a submission, or a collection
      // that frees a slot and memory)
      srv->adm.wait_admissible(srv->cv_work, lock, [&] { return srv->stop; });
      continue;
    }
    // wait for the oldest round; meanwhile admit arrivals, and go back to
    // enqueue the next one once the oldest is near its end and there is work
    Round& R = srv->rounds[srv->inflight.front()];
    stencil_status st = STENCIL_OK;
    bool completed = false;
    while (!srv->stop) {
      const hipError_t q = hipEventQuery(R.done);
      if (q == hipSuccess) {
        completed = true;
        break;
      }
      if (q != hipErrorNotReady) {
        st = hip_fail(q, "server round");
        break;
      }
      admit_locked(srv);
      reap_uploads_locked(srv);
      if (compose_now(srv) && std::any_of(srv->adm.resident.begin(), srv->adm.resident.end(), schedulable))
        break;
      srv->cv_work.wait_for(lock, std::chrono::microseconds(100));
    }
    if (st == STENCIL_OK && completed && *R.report != 0u) st = STENCIL_ERR_TIMEOUT;
    if (st != STENCIL_OK) {
      fail_inflight(srv, lock, st);
      continue;
    }
    if (completed) retire_round(srv);
  }
}

// Give back a collected (or dropped) request's device memory. mu held.
void release_locked(stencil_server_s* srv, Request* r) {
  if (srv->adm.release(r)) srv->st.hbm_in_use = srv->adm.in_use;
  if (r->dev) {
    // the block may still be the target of an admission copy that no round
    // waited for (a request that failed before its first round)
    if (hipEventRecord(srv->copy_mark, srv->copy) == hipSuccess)
      (void)hipStreamWaitEvent(srv->collect, srv->copy_mark, 0);
    (void)hipFreeAsync(r->dev, srv->collect);
  }
  r->dev = nullptr;
  if (r->host_in) {
    // the admission copy may still be in flight for a request that never ran
    (void)hipStreamSynchronize(srv->copy);
    srv->pinned.put(r->host_in, r->host_cls);
    r->host_in = nullptr;
  }
  srv->cv_work.notify_all();  // a slot and memory are free again
}

stencil_status collect(stencil_server_s* srv, uint64_t ticket, void* host_out, bool block,
                       int32_t* done, double* latency_s) {
  std::unique_lock<std::mutex> lock(srv->mu);
  auto it = srv->all.find(ticket);
  if (it == srv->all.end()) return fail(STENCIL_ERR_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
  Request* r = it->second.get();
  if (block)
    srv->cv_done.wait(lock, [&] { return r->state == RState::kDone || r->state == RState::kFailed; });
  if (r->state != RState::kDone && r->state != RState::kFailed) {
    if (done) *done = 0;
    return STENCIL_OK;
  }
  if (r->collecting) return fail(STENCIL_ERR_INVALID, "ticket %llu is being collected", (unsigned long long)ticket);
  if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
  stencil_status st = r->err;
  if (st == STENCIL_OK && host_out) {
    // the round that finished the request is complete; copy on the collect
    // stream without holding the scheduler's lock
    r->collecting = true;
    const void* src = r->grid(r->cur);
    const size_t bytes = r->bytes;
    lock.unlock();
    hipError_t e;
    {
      // device -> pinned bounce block by DMA, then a host copy
      std::lock_guard<std::mutex> cl(srv->collect_mu);
      size_t cls = 0;
      void* bounce = srv->pinned.get(bytes, &cls);
      if (!bounce) {
        e = hipErrorOutOfMemory;
      } else {
        e = hipMemcpyAsync(bounce, src, bytes, hipMemcpyDeviceToHost, srv->collect);
        if (e == hipSuccess) e = hipStreamSynchronize(srv->collect);
        if (e == hipSuccess) staging_copy(host_out, bounce, bytes);
        srv->pinned.put(bounce, cls);
      }
    }
    lock.lock();
    if (e != hipSuccess) st = hip_fail(e, "server result copy");
  }
  release_locked(srv, r);
  srv->all.erase(it);
  if (done) *done = 1;
  return st == STENCIL_OK ? STENCIL_OK : fail(st, "request %llu failed", (unsigned long long)ticket);
}

}  // namespace

extern "C" {

stencil_status stencil_server_create(const stencil_server_config* config, stencil_server_t* server) {
  if (!config || !server) return fail(STENCIL_ERR_INVALID, "NULL argument");
  *server = nullptr;
  if (config->max_slots < 1) return fail(STENCIL_ERR_INVALID, "max_slots must be >= 1");
  if (config->hbm_budget_bytes == 0) return fail(STENCIL_ERR_INVALID, "HBM budget must be > 0");
  if (config->rounds_in_flight > kMaxRoundsInFlight)
    return fail(STENCIL_ERR_INVALID, "rounds_in_flight must be 1 or 2");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || config->device < 0 || config->device >= ndev)
    return fail(STENCIL_ERR_DEVICE, "HIP device %d is not available", config->device);
  std::unique_ptr<stencil_server_s> srv(new (std::nothrow) stencil_server_s());
  if (!srv) return fail(STENCIL_ERR_NOMEM, "host allocation failed");
  srv->cfg = *config;
  srv->adm.budget = config->hbm_budget_bytes;
  srv->adm.slots = config->max_slots;
  if (srv->cfg.rounds_in_flight <= 0) srv->cfg.rounds_in_flight = 1;
  if (srv->cfg.quantum_passes <= 0) srv->cfg.quantum_passes = 4;
  if (!(srv->cfg.round_target_s > 0)) srv->cfg.round_target_s = 0.0;
  std::memset(&srv->st, 0, sizeof(srv->st));
  int prev = 0;
  (void)hipGetDevice(&prev);
  hipError_t e = hipSetDevice(config->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&srv->compute, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&srv->copy, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&srv->collect, hipStreamNonBlocking);
  for (int k = 0; k < kMaxRoundsInFlight && e == hipSuccess; ++k) {
    e = hipEventCreateWithFlags(&srv->rounds[k].done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc((void**)&srv->rounds[k].report, sizeof(unsigned int), hipHostMallocDefault);
    if (e == hipSuccess) *srv->rounds[k].report = 0u;
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&srv->inputs_ready, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&srv->copy_mark, hipEventDisableTiming);
  if (e == hipSuccess) {
    hipMemPoolProps props;
    std::memset(&props, 0, sizeof(props));
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = config->device;
    e = hipMemPoolCreate(&srv->pool, &props);
    uint64_t keep = config->hbm_budget_bytes;
    if (e == hipSuccess) e = hipMemPoolSetAttribute(srv->pool, hipMemPoolAttrReleaseThreshold, &keep);
  }
  (void)hipSetDevice(prev);
  if (e != hipSuccess) {
    stencil_server_destroy(srv.release());
    return hip_fail(e, "server streams");
  }
  stencil_server_s* raw = srv.release();
  raw->worker = std::thread(scheduler, raw);
  *server = raw;
  return STENCIL_OK;
}

stencil_status stencil_server_submit(stencil_server_t srv, const stencil_job* job, const void* host_in,
                                     uint64_t* ticket) {
  if (!srv || !job || !host_in || !ticket) return fail(STENCIL_ERR_INVALID, "NULL argument");
  // latency counts from the call, so planning and host staging are inside it
  const Clock::time_point t_call = Clock::now();
  // planned as a round's batch plans it: the depth found here is the one
  // every round then runs the request at
  stencil_plan_t pl = nullptr;
  stencil_status st = plan_batch_job(*job, serve_seg_2d(), serve_seg_3d(), &pl);
  if (st != STENCIL_OK) {
    std::lock_guard<std::mutex> lock(srv->mu);
    srv->st.rejected++;
    return st;
  }
  std::unique_ptr<Request> r(new (std::nothrow) Request());
  if (!r) {
    stencil_plan_destroy(pl);
    return fail(STENCIL_ERR_NOMEM, "host allocation failed");
  }
  r->bytes = (size_t)pl->padded_elems * pl->elem;
  // two resident grids plus the batch workspaces of the rounds in flight
  r->need = (2 + (size_t)srv->cfg.rounds_in_flight) * align256(r->bytes);
  r->remaining = job->T;
  r->unscheduled = job->T;
  r->updates = (double)pl->cells * (double)job->T;
  r->depth = pl->scheme == STENCIL_SCHEME_NAIVE ? 1 : std::max(1, pl->depth);
  r->cells = std::max<int64_t>(1, pl->cells);
  r->plan.reset(pl);
  if (r->need > srv->cfg.hbm_budget_bytes) {
    std::lock_guard<std::mutex> lock(srv->mu);
    srv->st.rejected++;
    return fail(STENCIL_ERR_BUDGET, "request needs %zu bytes of device memory; the budget is %llu",
                r->need, (unsigned long long)srv->cfg.hbm_budget_bytes);
  }
  r->host_in = srv->pinned.get(r->bytes, &r->host_cls);
  if (!r->host_in) return fail(STENCIL_ERR_NOMEM, "pinned staging of %zu bytes failed", r->bytes);
  staging_copy(r->host_in, host_in, r->bytes);
  std::lock_guard<std::mutex> lock(srv->mu);
  r->ticket = srv->next_ticket++;
  r->t_submit = t_call;
  if (!srv->any_submit) {
    srv->any_submit = true;
    srv->first_submit = r->t_submit;
  }
  *ticket = r->ticket;
  srv->adm.queue.push_back(r.get());
  srv->all[r->ticket] = std::move(r);
  srv->st.submitted++;
  srv->st.queued = (int32_t)srv->adm.queue.size();
  srv->cv_work.notify_all();
  return STENCIL_OK;
}

stencil_status stencil_server_poll(stencil_server_t srv, uint64_t ticket, void* host_out, int32_t* done,
                                   double* latency_s) {
  if (!srv || !done) return fail(STENCIL_ERR_INVALID, "NULL argument");
  return collect(srv, ticket, host_out, false, done, latency_s);
}

stencil_status stencil_server_wait(stencil_server_t srv, uint64_t ticket, void* host_out, double* latency_s) {
  if (!srv) return fail(STENCIL_ERR_INVALID, "NULL argument");
  int32_t done = 0;
  return collect(srv, ticket, host_out, true, &done, latency_s);
}

stencil_status stencil_server_stats(stencil_server_t srv, stencil_server_statistics* out) {
  if (!srv || !out) return fail(STENCIL_ERR_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lock(srv->mu);
  *out = srv->st;
  std::vector<double> l = srv->latencies;
  std::sort(l.begin(), l.end());
  auto rank = [&](double p) {
    const size_t k = (size_t)std::ceil(p * (double)l.size());
    return l[std::min(l.size() - 1, k == 0 ? 0 : k - 1)];
  };
  if (!l.empty()) {
    out->p50_s = rank(0.50);
    out->p99_s = rank(0.99);
    out->max_s = l.back();
    double sum = 0;
    for (double v : l) sum += v;
    out->mean_s = sum / (double)l.size();
    out->wall_s = std::chrono::duration<double>(srv->last_done - srv->first_submit).count();
  }
  return STENCIL_OK;
}

stencil_status stencil_server_destroy(stencil_server_t srv) {
  if (!srv) return fail(STENCIL_ERR_INVALID, "NULL argument");
  {
    std::lock_guard<std::mutex> lock(srv->mu);
    srv->stop = true;
    srv->adm.queue.clear();
  }
  srv->cv_work.notify_all();
  if (srv->worker.joinable()) srv->worker.join();
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(srv->cfg.device);
  if (srv->compute) (void)hipStreamSynchronize(srv->compute);
  if (srv->copy) (void)hipStreamSynchronize(srv->copy);
  for (Upload& u : srv->uploads) (void)hipEventDestroy(u.done);
  srv->uploads.clear();
  for (auto& kv : srv->all) {
    if (kv.second->dev) (void)hipFreeAsync(kv.second->dev, srv->collect);
    srv->pinned.put(kv.second->host_in, kv.second->host_cls);  // freed with the pool
    kv.second->host_in = nullptr;
  }
  if (srv->collect) (void)hipStreamSynchronize(srv->collect);
  for (int k = 0; k < kMaxRoundsInFlight; ++k) {
    if (srv->rounds[k].done) (void)hipEventDestroy(srv->rounds[k].done);
    if (srv->rounds[k].report) (void)hipHostFree(srv->rounds[k].report);
  }
  if (srv->inputs_ready) (void)hipEventDestroy(srv->inputs_ready);
  if (srv->copy_mark) (void)hipEventDestroy(srv->copy_mark);
  if (srv->compute) (void)hipStreamDestroy(srv->compute);
  if (srv->copy) (void)hipStreamDestroy(srv->copy);
  if (srv->collect) (void)hipStreamDestroy(srv->collect);
  // every allocation from the pool has been freed and its stream drained
  if (srv->pool) (void)hipMemPoolDestroy(srv->pool);
  (void)hipSetDevice(prev);
  delete srv;
  return STENCIL_OK;
}

}  // extern "C"
