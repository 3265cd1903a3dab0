// Serving loop (see server.hip).
#pragma once

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <exception>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "solver.h"

namespace arr {

// First-fit allocator of offsets inside the server's device arena.
struct Arena {
  char *base = nullptr;
  size_t cap = 0;
  std::map<size_t, size_t> free_;  // offset -> bytes, coalesced
  bool alloc(size_t bytes, size_t &off);
  void release(size_t off, size_t bytes);
  size_t largest_free() const;
};

// The running requests' filter SpMMs, launched together. Each request's
// thread hands in one filter application at a time (a chain of SpMM calls,
// each depending on the one before) and blocks only until the chain is
// enqueued. The broker thread runs rounds on its stream: each round takes
// the next call of every chain in hand, as one multi-request launch per
// kernel variant (SpmmBatch; grid-form calls as launches of their own), so
// requests that filter at the same time advance in lockstep, and chains
// handed in meanwhile join at the next round. The broker's stream waits for
// a request's stream before its chain's first round; the request's stream
// waits for the chain's last round. Nothing on the device waits for a later
// submission, so no request can block another's progress.
class SpmmBroker {
 public:
  explicit SpmmBroker(int device);
  ~SpmmBroker();
  // For one request's thread: enqueues `calls` (in order) and orders s after
  // them (in_ev and done_ev are the request's own events).
  void submit(std::vector<std::function<void(hipStream_t)>> &calls, hipStream_t s, hipEvent_t in_ev,
              hipEvent_t done_ev);
  int64_t batches() const { return batches_.load(); }
  int64_t launches() const { return launches_.load(); }

 private:
  struct Item {
    std::vector<std::function<void(hipStream_t)>> *calls;
    size_t next = 0;
    hipEvent_t in_ev, done_ev;
    bool enqueued = false;
    std::exception_ptr err;
  };
  void loop();
  int device_;
  hipStream_t bs_ = nullptr;
  std::unique_ptr<SpmmBatch> batch_;
  std::mutex mu_;
  std::condition_variable cv_;
  std::vector<Item *> pending_;
  bool stop_ = false;
  std::atomic<int64_t> batches_{0}, launches_{0};
  std::thread th_;
};

class Server {
 public:
  explicit Server(const arr_server_opts_t &o);
  ~Server();
  uint64_t submit(Solver *s);
  bool poll(uint64_t id, int *status);
  int wait(uint64_t id, std::string *error);
  void times(uint64_t id, double *t_submit, double *t_admit, double *t_done);
  void batch_stats(int64_t *batches, int64_t *launches) const {
    *batches = broker_ ? broker_->batches() : 0;
    *launches = broker_ ? broker_->launches() : 0;
  }

 private:
  struct Request {
    Solver *solver = nullptr;
    size_t bytes = 0, off = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int status = 0;
    bool done = false;
    std::string error;
  };
  void schedule();
  void work(uint64_t id);
  double now() const;

  arr_server_opts_t o_;
  DevBuf arena_mem_;
  Arena arena_;
  int slots_ = 4, active_ = 0;
  bool stopping_ = false;
  uint64_t next_id_ = 1;
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<uint64_t> queue_;
  std::map<uint64_t, Request> reqs_;
  std::thread sched_;
  std::map<uint64_t, std::thread> workers_;  // running (or finished, not yet joined) requests
  std::vector<uint64_t> finished_;            // workers done with their request, to be joined
  std::chrono::steady_clock::time_point t0_;
  std::unique_ptr<SpmmBroker> broker_;  // null unless o_.batch_spmm
};

}  // namespace arr
