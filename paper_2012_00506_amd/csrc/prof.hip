// Launch timing registry (fb_profile_enable / fb_profile_read).
#include <mutex>
#include <vector>

#include "prof.h"

namespace fb {

namespace {
struct Pending {
  int cls;
  hipEvent_t a, b;
  double work;
};
struct Registry {
  std::mutex mu;
  bool on = false;
  std::vector<Pending> pending;
  int64_t launches[FB_PROF_NCLASS] = {};
  double ms[FB_PROF_NCLASS] = {};
  double work[FB_PROF_NCLASS] = {};
};
Registry& reg() {
  static Registry r;
  return r;
}
void collect_locked(Registry& r) {
  for (auto& p : r.pending) {
    float t = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
      r.launches[p.cls] += 1;
      r.ms[p.cls] += t;
      r.work[p.cls] += p.work;
    }
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  r.pending.clear();
}
}  // namespace

ProfScope::ProfScope(int c, hipStream_t s, double w) : cls(c), st(s), work(w) {
  Registry& r = reg();
  if (!r.on) return;
  // launches recorded into a graph are not timed one by one
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    a = b = nullptr;
    return;
  }
  (void)hipEventRecord(a, st);
}

ProfScope::~ProfScope() {
  if (!a) return;
  (void)hipEventRecord(b, st);
  Registry& r = reg();
  std::lock_guard<std::mutex> g(r.mu);
  r.pending.push_back({cls, a, b, work});
  if (r.pending.size() > 4096) collect_locked(r);
}

void prof_add_work(int cls, double work) {
  Registry& r = reg();
  std::lock_guard<std::mutex> g(r.mu);
  if (r.on && cls >= 0 && cls < FB_PROF_NCLASS) r.work[cls] += work;
}

}  // namespace fb

using namespace fb;

extern "C" int fb_profile_enable(int32_t on) {
  Registry& r = reg();
  std::lock_guard<std::mutex> g(r.mu);
  collect_locked(r);
  for (int i = 0; i < FB_PROF_NCLASS; ++i) {
    r.launches[i] = 0;
    r.ms[i] = 0.0;
    r.work[i] = 0.0;
  }
  r.on = on != 0;
  return 0;
}

extern "C" int fb_profile_read(int32_t cls, int64_t* launches, double* ms, double* work) {
  if (cls < 0 || cls >= FB_PROF_NCLASS) return -1;
  Registry& r = reg();
  std::lock_guard<std::mutex> g(r.mu);
  collect_locked(r);
  if (launches) *launches = r.launches[cls];
  if (ms) *ms = r.ms[cls];
  if (work) *work = r.work[cls];
  return 0;
}
