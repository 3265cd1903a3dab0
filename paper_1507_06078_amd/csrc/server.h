// Serving loop (see server.hip).
#pragma once

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
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

class Server {
 public:
  explicit Server(const arr_server_opts_t &o);
  ~Server();
  uint64_t submit(Solver *s);
  bool poll(uint64_t id, int *status);
  int wait(uint64_t id, std::string *error);
  void times(uint64_t id, double *t_submit, double *t_admit, double *t_done);

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
};

}  // namespace arr
