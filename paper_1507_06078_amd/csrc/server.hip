// Serving loop: continuous batching of eigensolve requests on one GPU.
//
//  * Admission by device footprint: the server owns one device arena (the
//    HBM budget, allocated once). A queued request is admitted, in strict
//    FIFO order, as soon as a solve slot is free and a contiguous arena block
//    of its exact footprint (Solver::footprint(): blocks, matrix, work) can be
//    carved out. Inside its block the request's solver bump-allocates (a
//    per-thread Pool), so no hipMalloc/hipFree -- which would synchronize the
//    whole device -- runs while other requests compute.
//  * Device-resident state: an admitted request keeps its CSR, iterate,
//    Krylov blocks and Ritz state in its block until it finishes; its results
//    are then copied to host memory and the block returns to the arena.
//  * Overlap: every admitted request runs its Algorithm 8 state machine in a
//    worker thread on its own HIP stream, so the kernels of different
//    requests execute concurrently; requests that arrive while others run join
//    as soon as a slot and memory free up.
//  * Multi-request SpMM (option batch_spmm, off by default): the running
//    requests' filter applications are handed to a broker thread, which runs
//    them in lockstep rounds, each round one multi-request launch per kernel
//    variant whose workgroups take the requests' workgroups from a device
//    task table (SpmmBroker). All SpMMs then share one stream; on a 64-request
//    mix the requests seldom filter at the same moment (most rounds hold one
//    request), and the serial stream costs more than the merged launches save
//    (25.2 s against 20.3 s), so by default each request launches its own
//    SpMMs and the device overlaps the requests' streams.
//  * Determinism: no kernel uses atomics in a reduction, and a request's
//    SpMM workgroups run the same code on the same rows whether launched
//    alone or in a multi-request launch, so a request's result does not
//    depend on what else is running.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

#include "server.h"

namespace arr {

bool Arena::alloc(size_t bytes, size_t &off) {
  bytes = (bytes + 255) / 256 * 256;
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second >= bytes) {
      off = it->first;
      const size_t rest = it->second - bytes;
      free_.erase(it);
      if (rest) free_[off + bytes] = rest;
      return true;
    }
  }
  return false;
}

void Arena::release(size_t off, size_t bytes) {
  bytes = (bytes + 255) / 256 * 256;
  auto it = free_.emplace(off, bytes).first;
  auto next = std::next(it);
  if (next != free_.end() && it->first + it->second == next->first) {
    it->second += next->second;
    free_.erase(next);
  }
  if (it != free_.begin()) {
    auto prev = std::prev(it);
    if (prev->first + prev->second == it->first) {
      prev->second += it->second;
      free_.erase(it);
    }
  }
}

size_t Arena::largest_free() const {
  size_t b = 0;
  for (auto &kv : free_) b = std::max(b, kv.second);
  return b;
}

SpmmBroker::SpmmBroker(int device) : device_(device) {
  ARR_HIP(hipSetDevice(device_));
  ARR_HIP(hipStreamCreateWithFlags(&bs_, hipStreamNonBlocking));
  // a round of 8 requests needs at most ~300 KB of task table
  batch_ = std::make_unique<SpmmBatch>((size_t)1 << 20);
  th_ = std::thread([this] { loop(); });
}

SpmmBroker::~SpmmBroker() {
  {
    std::unique_lock<std::mutex> lk(mu_);
    stop_ = true;
    cv_.notify_all();
  }
  if (th_.joinable()) th_.join();
  (void)hipStreamSynchronize(bs_);
  batch_.reset();
  (void)hipStreamDestroy(bs_);
}

void SpmmBroker::submit(std::vector<std::function<void(hipStream_t)>> &calls, hipStream_t s, hipEvent_t in_ev,
                        hipEvent_t done_ev) {
  if (calls.empty()) return;
  ARR_HIP(hipEventRecord(in_ev, s));  // the chain's inputs are ready here
  Item it;
  it.calls = &calls;
  it.in_ev = in_ev;
  it.done_ev = done_ev;
  {
    std::unique_lock<std::mutex> lk(mu_);
    ARR_REQUIRE(!stop_, "SpMM broker stopped");
    pending_.push_back(&it);
    cv_.notify_all();
    cv_.wait(lk, [&] { return it.enqueued; });
  }
  if (it.err) std::rethrow_exception(it.err);
  ARR_HIP(hipStreamWaitEvent(s, done_ev, 0));
}

void SpmmBroker::loop() {
  (void)hipSetDevice(device_);
  std::vector<Item *> active;  // chains with calls left, in arrival order
  std::unique_lock<std::mutex> lk(mu_);
  while (true) {
    if (active.empty()) cv_.wait(lk, [&] { return stop_ || !pending_.empty(); });
    std::vector<Item *> fresh;
    fresh.swap(pending_);
    if (active.empty() && fresh.empty()) break;  // stopping, nothing left
    lk.unlock();
    std::vector<Item *> done;
    try {
      for (Item *it : fresh) ARR_HIP(hipStreamWaitEvent(bs_, it->in_ev, 0));
      active.insert(active.end(), fresh.begin(), fresh.end());
      // one round: the next call of every chain
      struct Install {
        SpmmBatch *prev;
        explicit Install(SpmmBatch *b) : prev(spmm_batch()) { spmm_batch() = b; }
        ~Install() { spmm_batch() = prev; }
      };
      {
        Install in(batch_.get());
        for (Item *it : active) {
          try {
            (*it->calls)[it->next](bs_);
          } catch (...) {
            if (!it->err) it->err = std::current_exception();
          }
          ++it->next;
        }
      }
      launches_ += batch_->run(bs_);
      ++batches_;
      for (size_t q = 0; q < active.size();) {
        Item *it = active[q];
        if (it->next == it->calls->size()) {
          ARR_HIP(hipEventRecord(it->done_ev, bs_));
          done.push_back(it);
          active.erase(active.begin() + (long)q);
        } else {
          ++q;
        }
      }
    } catch (...) {
      // a failure outside one call's launches ends every chain in hand
      for (Item *it : active) {
        if (!it->err) it->err = std::current_exception();
        done.push_back(it);
      }
      active.clear();
    }
    lk.lock();
    for (Item *it : done) it->enqueued = true;
    if (!done.empty()) cv_.notify_all();
  }
}

Server::Server(const arr_server_opts_t &o) : o_(o) {
  t0_ = std::chrono::steady_clock::now();
  ARR_HIP(hipSetDevice(o.device));
  size_t budget = o.hbm_budget_bytes;
  if (budget == 0) {
    size_t fr = 0, tot = 0;
    ARR_HIP(hipMemGetInfo(&fr, &tot));
    budget = fr / 10 * 8;
  }
  budget = budget / 256 * 256;
  ARR_REQUIRE(budget > 0, "server: empty HBM budget");
  arena_mem_.alloc(budget);
  arena_.base = arena_mem_.as<char>();
  arena_.cap = budget;
  arena_.free_[0] = budget;
  slots_ = o.max_slots > 0 ? o.max_slots : 4;
  if (o.batch_spmm) broker_ = std::make_unique<SpmmBroker>(o.device);
  sched_ = std::thread([this] { schedule(); });
}

Server::~Server() {
  {
    std::unique_lock<std::mutex> lk(mu_);
    stopping_ = true;
    for (uint64_t id : queue_) {
      Request &r = reqs_[id];
      r.done = true;
      r.status = ARR_ESTATE;
      r.error = "cancelled: server destroyed before admission";
    }
    queue_.clear();
    cv_.notify_all();
  }
  if (sched_.joinable()) sched_.join();
  for (auto &kv : workers_)
    if (kv.second.joinable()) kv.second.join();
  broker_.reset();  // after every request that could hand it work
  // the handles outlive the server: drop their back-references
  for (auto &kv : reqs_)
    if (kv.second.solver && kv.second.solver->server == this) kv.second.solver->server = nullptr;
}

double Server::now() const {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count();
}

uint64_t Server::submit(Solver *s) {
  const size_t fp = s->footprint();
  ARR_REQUIRE(s->device() == o_.device, "handle was created for another device");
  if (fp > arena_.cap)
    throw Error(-2, "request footprint " + std::to_string(fp) + " bytes exceeds the server budget " +
                        std::to_string(arena_.cap));
  std::unique_lock<std::mutex> lk(mu_);
  ARR_REQUIRE(!stopping_, "server is shutting down");
  if (s->server) {
    ARR_REQUIRE(s->server == this, "handle is held by another server");
    auto it = reqs_.find(s->ticket);
    ARR_REQUIRE(it == reqs_.end() || it->second.done, "handle already has a request in flight");
  }
  const uint64_t id = next_id_++;
  Request &r = reqs_[id];
  r.solver = s;
  s->server = this;
  s->ticket = id;
  r.bytes = fp;
  r.t_submit = now();
  queue_.push_back(id);
  cv_.notify_all();
  return id;
}

void Server::schedule() {
  std::unique_lock<std::mutex> lk(mu_);
  // joins the threads of finished requests (their last step, under mu_, is
  // to list themselves; they take no lock after it)
  auto reap = [&] {
    for (uint64_t id : finished_) {
      auto it = workers_.find(id);
      if (it != workers_.end()) {
        if (it->second.joinable()) it->second.join();
        workers_.erase(it);
      }
    }
    finished_.clear();
  };
  while (true) {
    cv_.wait(lk, [&] { return stopping_ || !finished_.empty() || (!queue_.empty() && active_ < slots_); });
    reap();
    if (stopping_) break;
    if (queue_.empty() || active_ >= slots_) continue;
    Request &r = reqs_[queue_.front()];
    size_t off = 0;
    if (!arena_.alloc(r.bytes, off)) {
      // strict FIFO: the head waits until a running request returns memory
      cv_.wait(lk);
      continue;
    }
    const uint64_t id = queue_.front();
    queue_.pop_front();
    r.off = off;
    r.t_admit = now();
    ++active_;
    workers_.emplace(id, std::thread([this, id] { work(id); }));
  }
}

void Server::work(uint64_t id) {
  Solver *s;
  size_t off, bytes;
  {
    std::unique_lock<std::mutex> lk(mu_);
    Request &r = reqs_[id];
    s = r.solver;
    off = r.off;
    bytes = r.bytes;
  }
  int status = 0;
  std::string error;
  Pool pool;
  pool.base = arena_.base + off;
  pool.cap = bytes;
  // this request's SpMMs go to the broker (its events are created here, not
  // in the arena)
  struct BrokerSink : SpmmSink {
    SpmmBroker *b = nullptr;
    hipEvent_t in_ev = nullptr, done_ev = nullptr;
    std::vector<std::function<void(hipStream_t)>> calls;
    bool chain = false;
    void run(std::function<void(hipStream_t)> launch, hipStream_t st) override {
      calls.push_back(std::move(launch));
      if (!chain) flush(st);
    }
    void begin_chain() override { chain = true; }
    void end_chain(hipStream_t st) override {
      chain = false;
      flush(st);
    }
    void drop_chain() override {
      chain = false;
      calls.clear();
    }
    void flush(hipStream_t st) {
      std::vector<std::function<void(hipStream_t)>> c;
      c.swap(calls);
      b->submit(c, st, in_ev, done_ev);
    }
    ~BrokerSink() {
      // done_ev is recorded after every use of in_ev on the broker's stream
      if (done_ev) (void)hipEventSynchronize(done_ev);
      if (in_ev) (void)hipEventDestroy(in_ev);
      if (done_ev) (void)hipEventDestroy(done_ev);
    }
  } sink;
  try {
    ARR_HIP(hipSetDevice(o_.device));
    if (broker_) {
      sink.b = broker_.get();
      ARR_HIP(hipEventCreateWithFlags(&sink.in_ev, hipEventDisableTiming));
      ARR_HIP(hipEventCreateWithFlags(&sink.done_ev, hipEventDisableTiming));
      spmm_sink() = &sink;
    }
    device_pool() = &pool;
    s->ensure_device();
    status = s->solve();
    s->stash_results(s->keep_vectors());
  } catch (const Error &e) {
    status = e.code;
    error = e.what();
  } catch (const std::exception &e) {
    status = ARR_EDEVICE;
    error = e.what();
  }
  try {
    s->release_device();
  } catch (const std::exception &) {
  }
  device_pool() = nullptr;
  spmm_sink() = nullptr;
  std::unique_lock<std::mutex> lk(mu_);
  Request &r = reqs_[id];
  arena_.release(off, bytes);
  r.status = status;
  r.error = error;
  r.t_done = now();
  r.done = true;
  --active_;
  finished_.push_back(id);
  cv_.notify_all();
}

bool Server::poll(uint64_t id, int *status) {
  std::unique_lock<std::mutex> lk(mu_);
  auto it = reqs_.find(id);
  ARR_REQUIRE(it != reqs_.end(), "unknown ticket");
  if (it->second.done && status) *status = it->second.status;
  return it->second.done;
}

int Server::wait(uint64_t id, std::string *error) {
  std::unique_lock<std::mutex> lk(mu_);
  auto it = reqs_.find(id);
  ARR_REQUIRE(it != reqs_.end(), "unknown ticket");
  cv_.wait(lk, [&] { return it->second.done; });
  if (error) *error = it->second.error;
  return it->second.status;
}

void Server::times(uint64_t id, double *t_submit, double *t_admit, double *t_done) {
  std::unique_lock<std::mutex> lk(mu_);
  auto it = reqs_.find(id);
  ARR_REQUIRE(it != reqs_.end(), "unknown ticket");
  if (t_submit) *t_submit = it->second.t_submit;
  if (t_admit) *t_admit = it->second.t_admit;
  if (t_done) *t_done = it->second.t_done;
}

}  // namespace arr
