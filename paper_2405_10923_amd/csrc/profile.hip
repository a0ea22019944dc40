// Per-kernel timing: rhqr_profile_begin / rhqr_profile_end.
//
// While profiling is on, every launch of a timed kernel takes a pair of HIP
// events that its own dispatch records (start and end of the kernel), so the
// durations exclude launch gaps.  The state is process-wide and guarded by a
// mutex; calls from several host threads are safe, but a profile window
// collects the launches of every thread.
#include "common.h"

#include <atomic>
#include <mutex>
#include <vector>

namespace {

struct Profile {
  std::mutex mu;
  std::atomic<bool> on{false};
  std::vector<hipEvent_t> ev;  // pairs (start, stop)
  std::vector<int> cls;        // class of each pair
  size_t used = 0;             // events handed out in this window
};

Profile &prof() {
  static Profile p;
  return p;
}

}  // namespace

int prof_events(int cls, hipEvent_t *e0, hipEvent_t *e1) {
  *e0 = nullptr;
  *e1 = nullptr;
  Profile &p = prof();
  if (!p.on.load(std::memory_order_acquire)) return RHQR_OK;
  std::lock_guard<std::mutex> lk(p.mu);
  if (!p.on.load(std::memory_order_relaxed)) return RHQR_OK;
  while (p.used + 2 > p.ev.size()) {
    hipEvent_t e;
    RHQR_HIP(hipEventCreate(&e));
    p.ev.push_back(e);
  }
  if (p.cls.size() < p.ev.size() / 2) p.cls.resize(p.ev.size() / 2);
  *e0 = p.ev[p.used];
  *e1 = p.ev[p.used + 1];
  p.cls[p.used / 2] = cls;
  p.used += 2;
  return RHQR_OK;
}

extern "C" int rhqr_profile_begin(void) {
  Profile &p = prof();
  std::lock_guard<std::mutex> lk(p.mu);
  p.used = 0;
  p.on.store(true, std::memory_order_release);
  return RHQR_OK;
}

extern "C" int rhqr_profile_end(int32_t nclass, double *h_ms, int64_t *h_launches) {
  if (nclass < 0 || nclass > RHQR_PROF_NCLASS) return -1;
  if (nclass > 0 && !h_ms) return -2;
  if (nclass > 0 && !h_launches) return -3;
  Profile &p = prof();
  std::lock_guard<std::mutex> lk(p.mu);
  p.on.store(false, std::memory_order_release);
  for (int c = 0; c < nclass; ++c) {
    h_ms[c] = 0.0;
    h_launches[c] = 0;
  }
  int rc = RHQR_OK;
  for (size_t k = 0; k + 1 < p.used; k += 2) {
    const int c = p.cls[k / 2];
    if (hipEventSynchronize(p.ev[k + 1]) != hipSuccess) {
      rc = RHQR_ERR_HIP;
      continue;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.ev[k], p.ev[k + 1]) != hipSuccess) {
      rc = RHQR_ERR_HIP;
      continue;
    }
    if (c >= 0 && c < nclass) {
      h_ms[c] += ms;
      h_launches[c] += 1;
    }
  }
  p.used = 0;
  return rc;
}
