// Per-kernel launch timing with HIP events (tracing subsystem).
//
// When enabled, every kernel launch made by the library is bracketed by two
// events recorded on the launch's own stream; tsim_trace_get() waits for
// them and reports, per kernel name, the launch count and total duration.
// Disabled (the default), a launch costs one branch.
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace {

struct Rec {
  const char *name;
  hipEvent_t a, b;
};

struct Agg {
  std::string name;
  double ms = 0.0;
  int n = 0;
};

std::mutex g_mu;
bool g_on = false;
thread_local int t_quiet = 0;  // > 0 inside a TraceQuiet scope: launches are not traced
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
std::vector<Agg> g_agg;

hipEvent_t take() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void fold() {
  // caller holds g_mu
  for (auto &r : g_recs) {
    float ms = 0.f;
    if (r.a && r.b && hipEventSynchronize(r.b) == hipSuccess &&
        hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      Agg *hit = nullptr;
      for (auto &g : g_agg)
        if (g.name == r.name) hit = &g;
      if (!hit) {
        g_agg.push_back(Agg{r.name, 0.0, 0});
        hit = &g_agg.back();
      }
      hit->ms += ms;
      hit->n += 1;
    }
    if (r.a) g_pool.push_back(r.a);
    if (r.b) g_pool.push_back(r.b);
  }
  g_recs.clear();
}

}  // namespace

TraceQuiet::TraceQuiet() { ++t_quiet; }
TraceQuiet::~TraceQuiet() { --t_quiet; }

TraceScope::TraceScope(const char *name, hipStream_t s) : s_(s), slot_(-1) {
  if (t_quiet > 0) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on) return;
  Rec r{name, take(), take()};
  if (!r.a || !r.b) return;
  if (hipEventRecord(r.a, s) != hipSuccess) return;
  slot_ = int(g_recs.size());
  g_recs.push_back(r);
}

TraceScope::~TraceScope() {
  if (slot_ < 0) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (slot_ < int(g_recs.size())) (void)hipEventRecord(g_recs[slot_].b, s_);
}

extern "C" {

int tsim_trace_enable(int on) {
  std::lock_guard<std::mutex> lk(g_mu);
  fold();
  g_agg.clear();
  g_on = on != 0;
  return TSIM_OK;
}

int tsim_trace_get(int index, char *name, size_t name_len, double *total_ms, int *launches) {
  if (!name || name_len == 0 || !total_ms || !launches) return TSIM_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  fold();
  if (index < 0 || index >= int(g_agg.size())) return TSIM_EINVAL;
  std::strncpy(name, g_agg[index].name.c_str(), name_len - 1);
  name[name_len - 1] = '\0';
  *total_ms = g_agg[index].ms;
  *launches = g_agg[index].n;
  return TSIM_OK;
}

int tsim_trace_count(int *n) {
  if (!n) return TSIM_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  fold();
  *n = int(g_agg.size());
  return TSIM_OK;
}

}  // extern "C"
