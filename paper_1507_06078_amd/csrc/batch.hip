// Host side of the multi-request filter SpMM (SpmmBatch, see common.h) and
// the thread-local hooks launch_filter_spmm consults: the batch that collects
// its launches and the sink that takes whole calls. The task kernel itself
// and the launchers the batch calls are in spmm.hip.
#include <algorithm>
#include <cstring>
#include <functional>

#include "common.h"

namespace arr {

SpmmBatch *&spmm_batch() {
  static thread_local SpmmBatch *b = nullptr;
  return b;
}

SpmmSink *&spmm_sink() {
  static thread_local SpmmSink *k = nullptr;
  return k;
}

SpmmBatch::SpmmBatch(size_t cap_bytes) : cap_(cap_bytes) {
  dev_.alloc(cap_);
  ARR_HIP(hipHostMalloc((void **)&host_, cap_ * kRing, hipHostMallocDefault));
  for (hipEvent_t &e : staged_) ARR_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
}

SpmmBatch::~SpmmBatch() {
  for (hipEvent_t e : staged_)
    if (e) {
      (void)hipEventSynchronize(e);
      (void)hipEventDestroy(e);
    }
  if (host_) (void)hipHostFree(host_);
}

void SpmmBatch::add(const SpmmTask &t, SpmmTaskLauncher launcher) {
  tasks_.push_back(t);
  launchers_.push_back(launcher);
}

int SpmmBatch::run(hipStream_t s) {
  const int nl = (int)tasks_.size();
  if (nl == 0) return 0;
  // the collected work is consumed whether or not the launch succeeds
  struct Forget {
    SpmmBatch *b;
    ~Forget() {
      b->tasks_.clear();
      b->launchers_.clear();
    }
  } forget{this};
  // launches of one kernel variant together; inside a variant, workgroup b of
  // every launch before workgroup b + 1 of any, so the persistent grid's
  // static deal mixes the requests
  std::vector<int> order(nl);
  for (int i = 0; i < nl; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return std::less<const void *>()((const void *)launchers_[a], (const void *)launchers_[b]);
  });
  std::vector<int2> pairs;
  std::vector<std::pair<SpmmTaskLauncher, std::pair<size_t, int>>> runs;  // launcher, (first pair, count)
  for (int i = 0; i < nl;) {
    int j = i;
    int gmax = 0;
    while (j < nl && launchers_[order[j]] == launchers_[order[i]]) gmax = std::max(gmax, tasks_[order[j++]].groups);
    const size_t first = pairs.size();
    for (int b = 0; b < gmax; ++b)
      for (int q = i; q < j; ++q)
        if (b < tasks_[order[q]].groups) pairs.push_back(int2{order[q], b});
    runs.push_back({launchers_[order[i]], {first, (int)(pairs.size() - first)}});
    i = j;
  }
  const size_t db = sizeof(SpmmTask) * nl, dpad = (db + 255) / 256 * 256, pb = sizeof(int2) * pairs.size();
  ARR_REQUIRE(dpad + pb <= cap_, "multi-request SpMM: task table exceeds its buffer");
  char *h = host_ + cap_ * slot_;
  ARR_HIP(hipEventSynchronize(staged_[slot_]));  // the copy kRing runs back has left this buffer
  std::memcpy(h, tasks_.data(), db);
  std::memcpy(h + dpad, pairs.data(), pb);
  ARR_HIP(hipMemcpyAsync(dev_.p, h, dpad + pb, hipMemcpyHostToDevice, s));
  ARR_HIP(hipEventRecord(staged_[slot_], s));
  slot_ = (slot_ + 1) % kRing;
  const SpmmTask *ddesc = (const SpmmTask *)dev_.p;
  const int2 *dpairs = (const int2 *)((const char *)dev_.p + dpad);
  for (auto &r : runs) r.first(ddesc, dpairs + r.second.first, r.second.second, s);
  ARR_HIP(hipGetLastError());
  return nl;
}

}  // namespace arr
