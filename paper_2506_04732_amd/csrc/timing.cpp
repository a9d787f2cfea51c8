// Optional per-kernel-class timing with HIP events (bench instrumentation).
#include <mutex>
#include <vector>

#include "common.h"

namespace t2s2 {

namespace {
struct Rec {
  int cls;
  hipEvent_t a, b;
  double bytes, flops;
};
struct TimingState {
  bool enabled = false;
  unsigned mask = ~0u;  // classes recorded while enabled
  std::vector<Rec> done;      // both recorded
  std::vector<hipEvent_t> pool;
  double ms[KC_COUNT] = {0}, bytes[KC_COUNT] = {0}, flops[KC_COUNT] = {0};
  long launches[KC_COUNT] = {0};
};
TimingState g_t;
std::mutex g_m;
// begin recorded, end pending: a stack per host thread, so that concurrent
// solves on several streams (batched solves) pair their own events
thread_local std::vector<Rec> t_open;

hipEvent_t take_event() {
  if (!g_t.pool.empty()) {
    hipEvent_t e = g_t.pool.back();
    g_t.pool.pop_back();
    return e;
  }
  hipEvent_t e;
  T2S2_HIP(hipEventCreate(&e));
  return e;
}

// fold completed records into the totals (blocking on their end events)
void drain() {
  for (auto& r : g_t.done) {
    T2S2_HIP(hipEventSynchronize(r.b));
    float ms = 0.f;
    T2S2_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    g_t.ms[r.cls] += ms;
    g_t.bytes[r.cls] += r.bytes;
    g_t.flops[r.cls] += r.flops;
    g_t.launches[r.cls] += 1;
    g_t.pool.push_back(r.a);
    g_t.pool.push_back(r.b);
  }
  g_t.done.clear();
}
}  // namespace

bool timing_enabled(int cls) { return g_t.enabled && (cls < 0 || ((g_t.mask >> cls) & 1u)); }

void timing_select(unsigned mask) {
  std::lock_guard<std::mutex> lk(g_m);
  g_t.mask = mask;
}

void timing_record_begin(hipStream_t s, int cls, double bytes, double flops) {
  std::lock_guard<std::mutex> lk(g_m);
  Rec r{cls, take_event(), take_event(), bytes, flops};
  T2S2_HIP(hipEventRecord(r.a, s));
  t_open.push_back(r);
}

void timing_record_end(hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_m);
  if (t_open.empty()) return;
  Rec r = t_open.back();
  t_open.pop_back();
  T2S2_HIP(hipEventRecord(r.b, s));
  g_t.done.push_back(r);
  if (g_t.done.size() >= 4096) drain();
}

void timing_set(bool on) {
  std::lock_guard<std::mutex> lk(g_m);
  drain();
  g_t.enabled = on;
  for (int i = 0; i < KC_COUNT; ++i) g_t.ms[i] = g_t.bytes[i] = g_t.flops[i] = 0.0, g_t.launches[i] = 0;
}

void timing_read(int cls, double* ms, long* launches, double* bytes, double* flops) {
  std::lock_guard<std::mutex> lk(g_m);
  drain();
  *ms = g_t.ms[cls];
  *launches = g_t.launches[cls];
  *bytes = g_t.bytes[cls];
  *flops = g_t.flops[cls];
}

}  // namespace t2s2
