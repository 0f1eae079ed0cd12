// Event-bracketed timing of named kernel regions (see prof.h).
#include "prof.h"

#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace zk {

namespace {

struct Region {
  std::string name;
  hipEvent_t a = nullptr, b = nullptr;
  bool closed = false;
};

std::atomic<bool> g_on{false};
std::mutex g_mu;
std::map<int, Region> g_regions;
int g_next = 0;
std::vector<hipEvent_t> g_pool;
std::string g_filter;  // empty: record every region

hipEvent_t take_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

}  // namespace

bool prof_enabled() { return g_on.load(std::memory_order_relaxed); }

void prof_set_enabled(bool on) { g_on.store(on); }

void prof_set_filter(const char* name) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_filter = name ? name : "";
}

ProfToken prof_begin(const char* name, hipStream_t s) {
  ProfToken t;
  if (!prof_enabled()) return t;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_filter.empty() && g_filter != name) return t;
  Region r;
  r.name = name;
  r.a = take_event();
  r.b = take_event();
  if (!r.a || !r.b || hipEventRecord(r.a, s) != hipSuccess) return t;
  t.id = g_next++;
  g_regions[t.id] = r;
  return t;
}

void prof_end(ProfToken t, hipStream_t s) {
  if (t.id < 0) return;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_regions.find(t.id);
  if (it == g_regions.end()) return;
  if (hipEventRecord(it->second.b, s) == hipSuccess) it->second.closed = true;
}

int prof_read(const char* name, double* total_ms, unsigned long long* count, bool reset) {
  std::lock_guard<std::mutex> lk(g_mu);
  double tot = 0;
  unsigned long long n = 0;
  for (auto it = g_regions.begin(); it != g_regions.end();) {
    Region& r = it->second;
    const bool match = r.closed && (std::strcmp(r.name.c_str(), name) == 0);
    if (match) {
      if (hipEventSynchronize(r.b) != hipSuccess) return -1;
      float ms = 0;
      if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return -1;
      tot += ms;
      n++;
    }
    if (reset && match) {
      g_pool.push_back(r.a);
      g_pool.push_back(r.b);
      it = g_regions.erase(it);
    } else {
      ++it;
    }
  }
  *total_ms = tot;
  *count = n;
  return 0;
}

}  // namespace zk
