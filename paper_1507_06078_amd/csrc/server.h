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

// The running requests' filter SpMMs, gathered and launched together: each
// request's thread hands its launch_filter_spmm calls in (through a
// per-request SpmmSink) and blocks only until they are enqueued; the broker
// thread takes whatever the running requests have handed in, makes its
// stream wait for each request's stream, runs all of it as one multi-request
// launch per kernel variant (SpmmBatch) and makes each request's stream wait
// for that launch. Nothing on the device waits for a later submission, so no
// request can block another's progress.
class SpmmBroker {
 public:
  explicit SpmmBroker(int device);
  ~SpmmBroker();
  // For one request's thread: runs `launch` in the next multi-request launch
  // and orders s after it (in_ev and done_ev are the request's own events).
  int submit(const std::function<int(hipStream_t)> &launch, hipStream_t s, hipEvent_t in_ev, hipEvent_t done_ev);
  int64_t batches() const { return batches_.load(); }
  int64_t launches() const { return launches_.load(); }

 private:
  struct Item {
    const std::function<int(hipStream_t)> *launch;
    hipEvent_t in_ev, done_ev;
    int result = 0;
    bool enqueued = false;
    std::exception_ptr err;
  };
  void loop();
  // rounds go to the streams in turn, so that consecutive rounds (of
  // requests that were not ready together) can still overlap on the device
  static constexpr int kStreams = 4;
  int device_;
  hipStream_t bs_[kStreams] = {};
  std::unique_ptr<SpmmBatch> batch_[kStreams];
  int next_ = 0;
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
