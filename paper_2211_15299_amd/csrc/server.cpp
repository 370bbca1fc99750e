// Continuous-batching request server for homogeneous-support DFTs.
//
// Clients submit (N, J, samples) requests from any thread and collect results
// by polling.  Three parts:
//   * a plan cache with a hard budget of device bytes: every byte of a
//     resident plan, of a plan being created and of an evicted plan not yet
//     freed counts against cfg.plan_bytes, which is never exceeded;
//   * a planner thread that creates the plans of requests whose support is
//     not resident (outside the cache lock, so clients and the scheduler never
//     wait for a plan upload), evicts least recently used plans that no
//     request holds, frees evicted plans itself (hipFree may wait for the
//     device), and holds a request back until its plan fits the budget;
//   * a scheduler thread that admits requests with resident plans into batch
//     slots in arrival order, runs each batch -- requests of different sizes
//     and supports -- as one grouped kernel launch that reads the samples and
//     writes the coefficients in pinned host memory mapped for the device,
//     and retires batches as the kernel signals their completion.
// A request holds a reference on its plan from admission to retirement, so
// a plan in use is never evicted.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hidft.h"
#include "internal.h"

namespace {

using Clock = std::chrono::steady_clock;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct PlanEntry {
  uint32_t M = 0;
  std::vector<uint64_t> J;
  uint64_t hash = 0;
  hidft_plan plan = nullptr;
  size_t bytes = 0;                // device bytes counted against the budget
  uint64_t refs = 0;               // admitted requests (queued or in flight)
  std::list<PlanEntry*>::iterator lru;
};

struct Request {
  uint64_t id = 0;
  PlanEntry* entry = nullptr;      // set once the plan is resident
  uint32_t M = 0;
  std::vector<uint64_t> J;         // kept only while the plan is not resident
  const float2* host_in = nullptr;
  float2* host_out = nullptr;
  uint64_t k = 0;
  uint32_t s = 0;
  Clock::time_point t_submit;
};

// Regions of a slot, in pinned host memory that the device reads and writes
// directly (mapped, coherent): the input region holds the batch's samples,
// then (from the next 256-byte boundary) its pack descriptors, then its
// instance descriptors; the output region the coefficients.  The grouped
// kernel loads the samples and stores the coefficients over the host link,
// so a batch is one launch and an event, with no copies.
struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  char* h_up = nullptr;            // samples | packs | instance descriptors
  float2* h_out = nullptr;         // coefficients of the batch
  char* d_up = nullptr;            // device addresses of h_up and h_out
  float2* d_out = nullptr;
  // Completion: the kernel's last block stores the batch's sequence number
  // to h_flag (mapped); d_count counts finished blocks over all launches.
  uint32_t* d_count = nullptr;
  uint32_t count_base = 0;
  uint32_t* h_flag = nullptr;
  uint32_t* d_flag = nullptr;
  uint32_t seq = 0;
  std::vector<Request> batch;      // requests in flight (empty when free)
  std::vector<uint64_t> offsets;   // point offset of each request in the region
  uint64_t points = 0;
};

// How long the scheduler keeps polling after its last launch or completion
// before it blocks on the request queue.
constexpr std::chrono::microseconds kSpinWindow{100};

// Host threads that share the scheduler's staging copies of a large batch
// (samples into the mapped region, coefficients out of it): one host thread
// copies about 17-20 GB/s, which bounds the server at about 10^6 requests/s
// when each of them is copied by the scheduler alone.  run() hands the
// copies out one request at a time, takes part itself and returns once all
// are done.  A helper registers (busy) under the lock under which run()
// publishes a generation, and run() waits for every helper to leave the
// previous one before it publishes the next, so a late helper never takes a
// copy of a finished generation.
class CopyPool {
 public:
  struct Job {
    void* dst;
    const void* src;
    size_t bytes;
  };
  void start(unsigned n_threads) {
    for (unsigned i = 0; i < n_threads; ++i) threads_.emplace_back([this] { work(); });
  }
  void stop() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : threads_) t.join();
    threads_.clear();
  }
  void run(const Job* jobs, size_t n) {
    while (busy_.load(std::memory_order_acquire) != 0) __builtin_ia32_pause();
    {
      std::lock_guard<std::mutex> lk(mu_);
      jobs_ = jobs;
      n_ = n;
      next_.store(0, std::memory_order_relaxed);
      done_.store(0, std::memory_order_relaxed);
      ++gen_;
    }
    cv_.notify_all();
    take(jobs, n);
    while (done_.load(std::memory_order_acquire) < n) __builtin_ia32_pause();
  }
  bool empty() const { return threads_.empty(); }

 private:
  void take(const Job* jobs, size_t n) {
    for (size_t i; (i = next_.fetch_add(1, std::memory_order_relaxed)) < n;) {
      std::memcpy(jobs[i].dst, jobs[i].src, jobs[i].bytes);
      done_.fetch_add(1, std::memory_order_release);
    }
  }
  void work() {
    uint64_t seen = 0;
    for (;;) {
      const Job* jobs;
      size_t n;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
        if (stop_) return;
        seen = gen_;
        jobs = jobs_;
        n = n_;
        busy_.fetch_add(1, std::memory_order_relaxed);
      }
      take(jobs, n);
      busy_.fetch_sub(1, std::memory_order_release);
    }
  }
  std::vector<std::thread> threads_;
  std::mutex mu_;
  std::condition_variable cv_;
  uint64_t gen_ = 0;
  bool stop_ = false;
  const Job* jobs_ = nullptr;
  size_t n_ = 0;
  std::atomic<size_t> next_{0}, done_{0};
  std::atomic<unsigned> busy_{0};
};

// Batches whose copies in one direction total at least this many bytes go
// through the pool; smaller ones (single requests at moderate load) are
// copied by the scheduler, with no hand-off latency.
constexpr size_t kPoolCopyBytes = 1u << 20;
constexpr unsigned kCopyHelpers = 3;

// Hash of a support for the plan cache: M, k and at most 64 entries of J
// spread over it (the first and the last included), so that a lookup costs
// O(1) here; find() compares the whole of J, which decides.
uint64_t hash_support(uint32_t M, const uint64_t* J, uint64_t k) {
  uint64_t h = 0x9e3779b97f4a7c15ULL ^ (M * 0x100000001b3ULL) ^ k;
  const uint64_t n = k < 64 ? k : 64;
  for (uint64_t i = 0; i < n; ++i) {
    const uint64_t j = J[n > 1 ? i * (k - 1) / (n - 1) : 0];
    h ^= j + 0x9e3779b97f4a7c15ULL + (h << 6) + (h >> 2);
  }
  return h;
}

}  // namespace

struct hidft_server_s {
  hidft_server_config cfg{};
  int device = -1;
  uint32_t grid = 0;               // blocks of the grouped kernel's persistent grid
  uint64_t slot_points = 0;        // complex values per slot and direction

  // plan cache (plan_mu)
  std::mutex plan_mu;
  std::condition_variable cv_plan;  // planner: work, or a plan reference dropped
  std::unordered_multimap<uint64_t, std::unique_ptr<PlanEntry>> plans;
  std::list<PlanEntry*> lru;       // front = most recently used
  std::deque<Request> need_plan;   // requests whose plan is not resident
  std::vector<std::pair<hidft_plan, size_t>> to_free;  // evicted, not yet freed
  size_t bytes_held = 0;           // resident + reserved + evicted-not-freed
  size_t bytes_peak = 0;
  bool planner_stop = false;
  hipStream_t plan_stream = nullptr;

  // requests (mu)
  std::mutex mu;
  std::condition_variable cv_work;   // scheduler: new requests or stop
  std::condition_variable cv_done;   // clients: results available
  std::deque<Request> pending;       // admitted (plan resident), not yet in a batch
  std::deque<hidft_server_result> results;
  uint64_t next_id = 1;
  uint64_t in_system = 0;            // submitted and not yet completed
  bool stop = false;

  std::vector<Slot> slots;
  std::thread worker, planner;
  CopyPool copies;                   // helpers of the scheduler's host copies
  std::vector<CopyPool::Job> jobs;   // the scheduler's copy list
  std::atomic<bool> planner_done{false};

  std::atomic<uint64_t> n_submitted{0}, n_completed{0}, n_rejected{0}, n_batches{0};
  std::atomic<uint64_t> n_plan_hits{0}, n_plan_misses{0}, n_plan_evictions{0};
  std::atomic<uint64_t> n_plan_waits{0}, n_failed{0};
  std::atomic<uint64_t> max_inflight{0};
  std::atomic<uint64_t> n_pending{0};  // requests queued and not yet in a batch
  std::atomic<int32_t> worker_error{0};

  void loop();
  void plan_loop();
  void launch(Slot& sl);
  void retire(Slot& sl);
  void copy_all(size_t bytes);
  PlanEntry* find(uint32_t M, const uint64_t* J, uint64_t k, uint64_t h);
  void admit(Request&& r);
  void fail_request(const Request& r, hidft_status st);
  void release(PlanEntry* e);
  hidft_status submit_batch(const hidft_server_request* reqs, uint64_t n, uint64_t* ids,
                            int32_t* statuses);
};

// The resident plan of (M, J), or null.  plan_mu held.
PlanEntry* hidft_server_s::find(uint32_t M, const uint64_t* J, uint64_t k, uint64_t h) {
  auto range = plans.equal_range(h);
  for (auto it = range.first; it != range.second; ++it) {
    PlanEntry* e = it->second.get();
    if (e->M == M && e->J.size() == k && std::memcmp(e->J.data(), J, k * sizeof(uint64_t)) == 0)
      return e;
  }
  return nullptr;
}

// Queues a request whose plan reference is taken for the scheduler.
void hidft_server_s::admit(Request&& r) {
  r.J.clear();
  r.J.shrink_to_fit();
  {
    std::lock_guard<std::mutex> lk(mu);
    pending.push_back(std::move(r));
    n_pending.fetch_add(1, std::memory_order_release);
  }
  cv_work.notify_one();
}

// Completes a request that could not be planned, with its status.
void hidft_server_s::fail_request(const Request& r, hidft_status st) {
  hidft_server_result res;
  res.id = r.id;
  res.status = st;
  res.batch_size = 0;
  res.latency_us = std::chrono::duration<double, std::micro>(Clock::now() - r.t_submit).count();
  {
    std::lock_guard<std::mutex> lk(mu);
    results.push_back(res);
    in_system--;
  }
  n_failed++;
  n_completed++;
  cv_done.notify_all();
}

void hidft_server_s::release(PlanEntry* e) {
  bool freed;
  {
    std::lock_guard<std::mutex> lk(plan_mu);
    freed = --e->refs == 0;
  }
  if (freed) cv_plan.notify_one();
}

// The planner: resolves each queued request's plan, in arrival order.
void hidft_server_s::plan_loop() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(plan_mu);
  for (;;) {
    cv_plan.wait(lk, [&] { return planner_stop || !need_plan.empty(); });
    if (need_plan.empty()) break;  // stopping, nothing left
    Request r = std::move(need_plan.front());
    need_plan.pop_front();
    const uint64_t h = hash_support(r.M, r.J.data(), r.k);
    if (PlanEntry* e = find(r.M, r.J.data(), r.k, h)) {
      // created for an earlier request of the same support
      ++e->refs;
      lru.splice(lru.begin(), lru, e->lru);
      n_plan_hits++;
      r.entry = e;
      r.s = e->plan->core.s;
      lk.unlock();
      admit(std::move(r));
      lk.lock();
      continue;
    }
    const size_t need = hidft::plan_table_bytes(r.k);
    bool waited = false;
    for (;;) {
      // Evict least recently used plans that no request holds, until the new
      // plan fits once they are freed.
      size_t freeing = 0;
      for (auto it = lru.end(); bytes_held - freeing + need > cfg.plan_bytes && it != lru.begin();) {
        --it;
        PlanEntry* v = *it;
        if (v->refs != 0) continue;
        to_free.emplace_back(v->plan, v->bytes);
        freeing += v->bytes;
        it = lru.erase(it);
        auto rg = plans.equal_range(v->hash);
        for (auto pi = rg.first; pi != rg.second; ++pi)
          if (pi->second.get() == v) {
            plans.erase(pi);  // frees v
            break;
          }
        n_plan_evictions++;
      }
      if (!to_free.empty()) {
        // Free outside the lock (hipFree may wait for the device), then scan
        // again: references may have dropped meanwhile.
        std::vector<std::pair<hidft_plan, size_t>> fr;
        fr.swap(to_free);
        lk.unlock();
        for (auto& p : fr) hidft_plan_destroy(p.first);
        lk.lock();
        for (auto& p : fr) bytes_held -= p.second;
        continue;
      }
      if (bytes_held + need <= cfg.plan_bytes) break;
      // Every resident plan is held by an admitted request, and the scan above
      // ran under the lock that release() takes: wait for the next reference
      // to drop (each admitted request retires, so this wait ends).
      if (!waited) n_plan_waits++;
      waited = true;
      cv_plan.wait(lk);
    }
    bytes_held += need;  // reserved for the plan being created
    bytes_peak = std::max(bytes_peak, bytes_held);
    lk.unlock();
    hidft_plan p = nullptr;
    const hidft_status st = hidft_plan_create(r.M, r.J.data(), r.k, 0, plan_stream, &p);
    lk.lock();
    if (st != HIDFT_OK) {
      bytes_held -= need;
      lk.unlock();
      fail_request(r, st);
      lk.lock();
      continue;
    }
    n_plan_misses++;
    auto owned = std::make_unique<PlanEntry>();
    PlanEntry* e = owned.get();
    e->M = r.M;
    e->J = r.J;
    e->hash = h;
    e->plan = p;
    e->bytes = need;
    e->refs = 1;
    lru.push_front(e);
    e->lru = lru.begin();
    plans.emplace(h, std::move(owned));
    r.entry = e;
    r.s = p->core.s;
    lk.unlock();
    admit(std::move(r));
    lk.lock();
  }
  planner_done.store(true, std::memory_order_release);
  lk.unlock();
  cv_work.notify_all();
}

// Runs the copies of `jobs` (`bytes` in all): through the pool when large.
void hidft_server_s::copy_all(size_t bytes) {
  if (bytes >= kPoolCopyBytes && jobs.size() > 1 && !copies.empty()) {
    copies.run(jobs.data(), jobs.size());
    return;
  }
  for (const CopyPool::Job& j : jobs) std::memcpy(j.dst, j.src, j.bytes);
}

// Stages the batch in `sl` and issues the grouped transform.
void hidft_server_s::launch(Slot& sl) {
  std::vector<std::pair<uint32_t, hidft::GroupSlot>> inst;
  inst.reserve(sl.batch.size());
  sl.offsets.resize(sl.batch.size());
  uint64_t off = 0;
  float2* d_in = reinterpret_cast<float2*>(sl.d_up);
  float2* d_out = sl.d_out;
  float2* h_in = reinterpret_cast<float2*>(sl.h_up);
  jobs.clear();
  for (size_t i = 0; i < sl.batch.size(); ++i) {
    const Request& r = sl.batch[i];
    sl.offsets[i] = off;
    jobs.push_back({h_in + off, r.host_in, r.k * sizeof(float2)});
    hidft::GroupSlot d;
    d.in = d_in + off;
    d.out = d_out + off;
    d.tw = r.entry->plan->d_tw;
    d.src = r.entry->plan->d_src;
    d.scale = r.entry->plan->scale;
    inst.emplace_back(r.s, d);
    off += r.k;
  }
  sl.points = off;
  copy_all(off * sizeof(float2));
  hipError_t e;
  const hidft::GroupDone done{sl.d_count, &sl.count_base, sl.d_flag, ++sl.seq};
  if (inst.size() <= hidft::GROUP_FEW_MAX) {
    // A few requests (most batches at moderate load): one block each, their
    // descriptors with the launch, no table staged.
    hidft::GroupFew few{};
    for (size_t i = 0; i < inst.size(); ++i) {
      few.slot[i] = inst[i].second;
      few.code[i] = inst[i].first | hidft::GROUP_SKIP_IDLE;
    }
    if ((e = hidft::launch_grouped_few(few, (uint32_t)inst.size(), sl.stream, &done)) !=
            hipSuccess ||
        (e = hipEventRecord(sl.done, sl.stream)) != hipSuccess) {
      worker_error = (int32_t)HIDFT_ERR_DEVICE;
    }
    n_batches++;
    return;
  }
  hidft::GroupSchedule sch;
  hidft::pack_instances(inst, grid, false, false, &sch);
  // A batch is often a single request: let the empty slots' wavefronts idle.
  for (auto& pk : sch.packs) pk.log2_k |= hidft::GROUP_SKIP_IDLE;
  const size_t packs_at = align_up(off * sizeof(float2), 256);
  const size_t slots_at = align_up(packs_at + sch.packs.size() * sizeof(hidft::GroupPack), 64);
  const size_t lanes_at = slots_at + sch.slots.size() * sizeof(hidft::GroupSlot);
  std::memcpy(sl.h_up + packs_at, sch.packs.data(), sch.packs.size() * sizeof(hidft::GroupPack));
  std::memcpy(sl.h_up + slots_at, sch.slots.data(), sch.slots.size() * sizeof(hidft::GroupSlot));
  std::memcpy(sl.h_up + lanes_at, sch.lane_end.data(), sch.lane_end.size() * sizeof(uint32_t));
  if ((e = hidft::launch_grouped(reinterpret_cast<const hidft::GroupPack*>(sl.d_up + packs_at),
                                 sch.n_wide, sch.n_narrow(),
                                 reinterpret_cast<const hidft::GroupSlot*>(sl.d_up + slots_at),
                                 reinterpret_cast<const uint32_t*>(sl.d_up + lanes_at), sch.grid,
                                 sl.stream, &done)) != hipSuccess ||
      (e = hipEventRecord(sl.done, sl.stream)) != hipSuccess) {
    worker_error = (int32_t)HIDFT_ERR_DEVICE;
  }
  n_batches++;
}

// Hands the results of a completed batch to the clients and frees the slot.
void hidft_server_s::retire(Slot& sl) {
  const int32_t st = worker_error.load() ? worker_error.load() : (int32_t)HIDFT_OK;
  const auto now = Clock::now();
  if (st == HIDFT_OK) {
    jobs.clear();
    for (size_t i = 0; i < sl.batch.size(); ++i) {
      const Request& r = sl.batch[i];
      jobs.push_back({r.host_out, sl.h_out + sl.offsets[i], r.k * sizeof(float2)});
    }
    copy_all(sl.points * sizeof(float2));
  }
  std::vector<hidft_server_result> done;
  done.reserve(sl.batch.size());
  for (size_t i = 0; i < sl.batch.size(); ++i) {
    const Request& r = sl.batch[i];
    hidft_server_result res;
    res.id = r.id;
    res.status = st;
    res.batch_size = (uint32_t)sl.batch.size();
    res.latency_us = std::chrono::duration<double, std::micro>(now - r.t_submit).count();
    done.push_back(res);
    release(r.entry);
  }
  sl.batch.clear();
  {
    std::lock_guard<std::mutex> lk(mu);
    for (auto& r : done) results.push_back(r);
    in_system -= done.size();
  }
  n_completed += done.size();
  cv_done.notify_all();
}

void hidft_server_s::loop() {
  (void)hipSetDevice(device);
  const uint64_t cap_points = slot_points;
  auto last_progress = Clock::now();
  for (;;) {
    bool progressed = false;
    uint64_t inflight = 0;
    for (Slot& sl : slots) {
      if (sl.batch.empty()) continue;
      // The kernel's own completion flag is seen a few microseconds before
      // the event; the event still catches a launch that failed.
      if (__atomic_load_n(sl.h_flag, __ATOMIC_ACQUIRE) == sl.seq) {
        retire(sl);
        progressed = true;
        continue;
      }
      const hipError_t q = hipEventQuery(sl.done);
      if (q == hipSuccess) {
        retire(sl);
        progressed = true;
      } else if (q != hipErrorNotReady) {
        worker_error = (int32_t)HIDFT_ERR_DEVICE;
        (void)hipStreamSynchronize(sl.stream);
        retire(sl);
        progressed = true;
      } else {
        ++inflight;
      }
    }
    for (Slot& sl : slots) {
      if (!sl.batch.empty()) continue;
      if (n_pending.load(std::memory_order_acquire) == 0) break;
      {
        std::lock_guard<std::mutex> lk(mu);
        uint64_t pts = 0;
        while (!pending.empty() && sl.batch.size() < cfg.max_batch &&
               pts + pending.front().k <= cap_points) {
          pts += pending.front().k;
          sl.batch.push_back(std::move(pending.front()));
          pending.pop_front();
          n_pending.fetch_sub(1, std::memory_order_relaxed);
        }
      }
      if (sl.batch.empty()) break;
      launch(sl);
      ++inflight;
      progressed = true;
    }
    uint64_t m = max_inflight.load();
    while (inflight > m && !max_inflight.compare_exchange_weak(m, inflight)) {
    }
    if (progressed) {
      last_progress = Clock::now();
      continue;
    }
    // While batches are on the device, and for a short window after the last
    // launch or completion, poll again without sleeping: a sleep, or the
    // wake-up of a condition variable, adds several microseconds to every
    // latency.  Measured at 20 000 requests/s against 5 us sleeps: p50 33 ->
    // 25 us, p99 75-77 -> 52-68 us (a 1 ms window was no better).  The
    // scheduler thread keeps one host core busy while it polls.
    if (inflight > 0 || Clock::now() - last_progress < kSpinWindow) {
      for (int i = 0; i < 32; ++i) __builtin_ia32_pause();
      continue;
    }
    std::unique_lock<std::mutex> lk(mu);
    // Stop once the planner has handed over every request and none is left.
    if (stop && pending.empty() && planner_done.load(std::memory_order_acquire)) break;
    cv_work.wait_for(lk, std::chrono::milliseconds(2),
                     [&] { return stop || !pending.empty(); });
  }
}

// Submits n requests.  Per request: the checks that need no lock, then the
// plan lookups of all of them under one hold of plan_mu, the support checks
// of those without a resident plan, the queueing of all of them under one
// hold of mu (ids in submission order) and one wake-up of the scheduler.
// statuses[i] and ids[i] (0 when refused) are set per request; the return
// value is the status of the last refused request (HIDFT_OK if none), and
// its message is the thread's last error.
hidft_status hidft_server_s::submit_batch(const hidft_server_request* reqs, uint64_t n,
                                          uint64_t* ids, int32_t* statuses) {
  struct Prep {
    Request r;
    uint64_t h = 0;
    int32_t st = HIDFT_OK;
    bool to_plan = false;  // accepted without a resident plan
    std::string err;
  };
  std::vector<Prep> prep(n);
  const auto now = Clock::now();
  for (uint64_t i = 0; i < n; ++i) {
    const hidft_server_request& q = reqs[i];
    Prep& p = prep[i];
    ids[i] = 0;
    if (!q.J || !q.host_samples || !q.host_coefs) {
      p.st = HIDFT_ERR_INVALID_ARGUMENT;
      p.err = "hidft_server_submit: NULL argument";
      continue;
    }
    if (q.k == 0 || q.k > slot_points) {
      n_rejected++;
      p.st = HIDFT_ERR_OUT_OF_MEMORY;
      p.err = "hidft_server_submit: request larger than a batch slot's memory";
      continue;
    }
    if (hidft::plan_table_bytes(q.k) > cfg.plan_bytes) {
      n_rejected++;
      p.st = HIDFT_ERR_OUT_OF_MEMORY;
      p.err = "hidft_server_submit: the plan alone exceeds the plan-cache budget";
      continue;
    }
    p.r.M = q.log2_n;
    p.r.host_in = static_cast<const float2*>(q.host_samples);
    p.r.host_out = static_cast<float2*>(q.host_coefs);
    p.r.k = q.k;
    p.r.t_submit = now;
    p.h = hash_support(q.log2_n, q.J, q.k);
  }
  {
    std::lock_guard<std::mutex> lk(plan_mu);
    for (uint64_t i = 0; i < n; ++i) {
      Prep& p = prep[i];
      if (p.st != HIDFT_OK) continue;
      if (PlanEntry* e = find(reqs[i].log2_n, reqs[i].J, reqs[i].k, p.h)) {
        ++e->refs;
        lru.splice(lru.begin(), lru, e->lru);
        n_plan_hits++;
        p.r.entry = e;
        p.r.s = e->plan->core.s;
      }
    }
  }
  for (uint64_t i = 0; i < n; ++i) {
    Prep& p = prep[i];
    if (p.st != HIDFT_OK || p.r.entry) continue;
    // Not resident: validate now, so that support errors return here; the
    // planner creates the plan.
    const uint32_t M = reqs[i].log2_n;
    const uint64_t* J = reqs[i].J;
    const uint64_t k = reqs[i].k;
    uint64_t mask = 0;
    std::string err;
    hidft_status st = hidft::analyze_core(M, J, k, &mask, &err);
    if (st == HIDFT_OK && (k & (k - 1)) != 0) {
      st = HIDFT_ERR_SIZE_NOT_POW2;
      err = "k is not a power of two";
    } else if (st == HIDFT_OK &&
               (uint32_t)__builtin_popcountll(mask) != (uint32_t)__builtin_ctzll(k)) {
      st = HIDFT_ERR_NOT_HOMOGENEOUS;
      err = "J is not homogeneous";
    } else if (st == HIDFT_OK && __builtin_ctzll(k) > (int)HIDFT_MAX_LOG2_K_DEVICE) {
      st = HIDFT_ERR_UNSUPPORTED;
      err = "k exceeds the executor's limit";
    }
    if (st != HIDFT_OK) {
      n_rejected++;
      p.st = st;
      p.err = "hidft_server_submit: " + err;
      continue;
    }
    p.r.J.assign(J, J + k);
  }
  bool any_resident = false, any_planned = false;
  uint64_t accepted = 0;
  std::vector<PlanEntry*> to_release;
  {
    std::lock_guard<std::mutex> lk(mu);
    for (uint64_t i = 0; i < n; ++i) {
      Prep& p = prep[i];
      if (p.st != HIDFT_OK) continue;
      if (stop) {
        if (p.r.entry) to_release.push_back(p.r.entry);
        p.r.entry = nullptr;
        p.st = HIDFT_ERR_INVALID_ARGUMENT;
        p.err = "hidft_server_submit: server stopping";
        continue;
      }
      p.r.id = next_id++;
      ids[i] = p.r.id;
      in_system++;
      ++accepted;
      if (p.r.entry) {
        pending.push_back(std::move(p.r));
        n_pending.fetch_add(1, std::memory_order_release);
        any_resident = true;
      } else {
        p.to_plan = true;
        any_planned = true;
      }
    }
  }
  for (PlanEntry* e : to_release) release(e);
  n_submitted += accepted;
  if (any_resident) cv_work.notify_one();
  if (any_planned) {
    std::vector<Request> refused;
    {
      std::lock_guard<std::mutex> lk(plan_mu);
      for (uint64_t i = 0; i < n; ++i) {
        Prep& p = prep[i];
        if (!p.to_plan) continue;
        if (!planner_stop)
          need_plan.push_back(std::move(p.r));
        else
          refused.push_back(std::move(p.r));
      }
    }
    cv_plan.notify_one();
    for (const Request& r : refused) fail_request(r, HIDFT_ERR_INVALID_ARGUMENT);
  }
  hidft_status last = HIDFT_OK;
  const std::string* msg = nullptr;
  for (uint64_t i = 0; i < n; ++i) {
    statuses[i] = prep[i].st;
    if (prep[i].st != HIDFT_OK) {
      last = (hidft_status)prep[i].st;
      msg = &prep[i].err;
    }
  }
  return hidft::set_error(last, msg ? *msg : std::string());
}

extern "C" {

hidft_status hidft_server_create(const hidft_server_config* cfg, hidft_server* out) {
  if (!out || !cfg)
    return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT, "hidft_server_create: NULL argument");
  *out = nullptr;
  if (cfg->slots == 0 || cfg->max_batch == 0 || cfg->data_bytes < 2 * 16 * cfg->slots ||
      cfg->plan_bytes == 0)
    return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT,
                            "hidft_server_create: slots, max_batch, data_bytes and plan_bytes "
                            "must be positive");
  auto sv = std::make_unique<hidft_server_s>();
  sv->cfg = *cfg;
  hipError_t e = hipGetDevice(&sv->device);
  if (e != hipSuccess) return hidft::hip_error(e, "hidft_server_create");
  if ((e = hidft::grouped_grid(&sv->grid)) != hipSuccess)
    return hidft::hip_error(e, "hidft_server_create: grid");
  sv->slot_points = cfg->data_bytes / cfg->slots / (2 * sizeof(float2));
  if ((e = hipStreamCreateWithFlags(&sv->plan_stream, hipStreamNonBlocking)) != hipSuccess)
    return hidft::hip_error(e, "hidft_server_create: stream");
  sv->slots.resize(cfg->slots);
  for (Slot& sl : sv->slots) {
    const size_t data = sv->slot_points * sizeof(float2);
    // samples, then packs and instance descriptors (one pack per instance at
    // most) after their alignment padding, then the schedule's lane table
    const size_t up = align_up(data, 256) +
                      align_up((size_t)cfg->max_batch * sizeof(hidft::GroupPack), 64) +
                      (size_t)cfg->max_batch * sizeof(hidft::GroupSlot) +
                      (size_t)sv->grid * hidft::GROUP_NARROW_PER_BLOCK * sizeof(uint32_t);
    if ((e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming)) != hipSuccess ||
        (e = hipHostMalloc(&sl.h_up, up, hipHostMallocMapped | hipHostMallocCoherent)) !=
            hipSuccess ||
        (e = hipHostMalloc(&sl.h_out, data, hipHostMallocMapped | hipHostMallocCoherent)) !=
            hipSuccess ||
        (e = hipHostGetDevicePointer(reinterpret_cast<void**>(&sl.d_up), sl.h_up, 0)) !=
            hipSuccess ||
        (e = hipHostGetDevicePointer(reinterpret_cast<void**>(&sl.d_out), sl.h_out, 0)) !=
            hipSuccess ||
        (e = hipMalloc(&sl.d_count, sizeof(uint32_t))) != hipSuccess ||
        (e = hipMemset(sl.d_count, 0, sizeof(uint32_t))) != hipSuccess ||
        (e = hipHostMalloc(&sl.h_flag, sizeof(uint32_t),
                           hipHostMallocMapped | hipHostMallocCoherent)) != hipSuccess ||
        (e = hipHostGetDevicePointer(reinterpret_cast<void**>(&sl.d_flag), sl.h_flag, 0)) !=
            hipSuccess) {
      hidft_status st = hidft::hip_error(e, "hidft_server_create: slot resources");
      hidft_server_destroy(sv.release());
      return st;
    }
  }
  for (Slot& sl : sv->slots) *sl.h_flag = 0;  // no batch has completed
  hidft_server s = sv.release();
  try {
    s->copies.start(kCopyHelpers);
    s->planner = std::thread([s] { s->plan_loop(); });
    s->worker = std::thread([s] { s->loop(); });
  } catch (...) {
    hidft_server_destroy(s);
    return hidft::set_error(HIDFT_ERR_DEVICE, "hidft_server_create: cannot start the threads");
  }
  *out = s;
  return hidft::set_error(HIDFT_OK, "");
}

hidft_status hidft_server_submit(hidft_server s, uint32_t log2_n, const uint64_t* J, uint64_t k,
                                 const void* host_samples, void* host_coefs, uint64_t* id) {
  if (!s) return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT, "hidft_server_submit: NULL server");
  if (!id) return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT, "hidft_server_submit: NULL argument");
  const hidft_server_request q{log2_n, J, k, host_samples, host_coefs};
  int32_t st = HIDFT_OK;
  return s->submit_batch(&q, 1, id, &st);
}

hidft_status hidft_server_submit_many(hidft_server s, const hidft_server_request* reqs,
                                      uint64_t n, uint64_t* ids, int32_t* statuses,
                                      uint64_t* n_accepted) {
  if (!s || (n > 0 && (!reqs || !ids || !statuses)))
    return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT,
                            "hidft_server_submit_many: NULL argument");
  if (n > 0) (void)s->submit_batch(reqs, n, ids, statuses);
  uint64_t acc = 0;
  for (uint64_t i = 0; i < n; ++i) acc += statuses[i] == HIDFT_OK;
  if (n_accepted) *n_accepted = acc;
  return hidft::set_error(HIDFT_OK, "");
}

hidft_status hidft_server_poll(hidft_server s, hidft_server_result* out, uint32_t cap,
                               uint32_t* n, int32_t wait_us) {
  if (!s || !n || (!out && cap > 0))
    return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT, "hidft_server_poll: NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->results.empty() && wait_us > 0)
    s->cv_done.wait_for(lk, std::chrono::microseconds(wait_us),
                        [&] { return !s->results.empty(); });
  uint32_t m = 0;
  while (m < cap && !s->results.empty()) {
    out[m++] = s->results.front();
    s->results.pop_front();
  }
  *n = m;
  return hidft::set_error(HIDFT_OK, "");
}

hidft_status hidft_server_drain(hidft_server s) {
  if (!s) return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT, "hidft_server_drain: NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->in_system == 0; });
  const int32_t err = s->worker_error.load();
  return err ? hidft::set_error((hidft_status)err, "hidft_server_drain: a batch failed")
             : hidft::set_error(HIDFT_OK, "");
}

hidft_status hidft_server_get_stats(hidft_server s, hidft_server_stats* st) {
  if (!s || !st) return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT, "hidft_server_get_stats: NULL");
  st->submitted = s->n_submitted;
  st->completed = s->n_completed;
  st->rejected = s->n_rejected;
  st->batches = s->n_batches;
  st->plan_hits = s->n_plan_hits;
  st->plan_misses = s->n_plan_misses;
  st->plan_evictions = s->n_plan_evictions;
  st->max_inflight_batches = s->max_inflight;
  {
    std::lock_guard<std::mutex> lk(s->plan_mu);
    st->plan_bytes_resident = s->bytes_held;
    st->plans_resident = s->plans.size();
    st->plan_bytes_peak = s->bytes_peak;
    st->waiting_for_plan = s->need_plan.size();
  }
  st->slot_bytes = 2 * s->slot_points * sizeof(float2);
  st->plan_waits = s->n_plan_waits;
  st->failed = s->n_failed;
  return hidft::set_error(HIDFT_OK, "");
}

hidft_status hidft_server_destroy(hidft_server s) {
  if (!s) return hidft::set_error(HIDFT_OK, "");
  // New submissions are refused from here.  The planner hands over every
  // request already queued for a plan (the scheduler keeps running, so plans
  // held by admitted requests keep being released), then the scheduler
  // finishes the admitted ones.
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  {
    std::lock_guard<std::mutex> lk(s->plan_mu);
    s->planner_stop = true;
  }
  s->cv_plan.notify_all();
  if (s->planner.joinable()) s->planner.join();
  s->planner_done.store(true, std::memory_order_release);
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  s->copies.stop();
  for (Slot& sl : s->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.h_up) (void)hipHostFree(sl.h_up);
    if (sl.h_flag) (void)hipHostFree(sl.h_flag);
    if (sl.d_count) (void)hipFree(sl.d_count);
    if (sl.h_out) (void)hipHostFree(sl.h_out);
  }
  for (auto& kv : s->plans) hidft_plan_destroy(kv.second->plan);
  for (auto& p : s->to_free) hidft_plan_destroy(p.first);
  if (s->plan_stream) (void)hipStreamDestroy(s->plan_stream);
  delete s;
  return hidft::set_error(HIDFT_OK, "");
}

}  // extern "C"
