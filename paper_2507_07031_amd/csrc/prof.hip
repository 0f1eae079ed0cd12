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

// Issue-rate calibration of v_mad_u64_u32 (the Montgomery products' only
// multiply): 8 independent dependent chains per thread, each step
// acc = lo32(acc) * b + acc, so the compiler can neither fold nor hoist the
// products.  MAD_UNROLL * 8 products per thread per iteration.
constexpr uint32_t MAD_UNROLL = 16;

__global__ __launch_bounds__(256) void mad_rate_kernel(uint32_t iters, uint32_t seed, uint32_t* sink) {
  uint64_t acc[8];
  const uint32_t b = seed ^ (threadIdx.x * 2654435761u) ^ 1u;
#pragma unroll
  for (int k = 0; k < 8; k++) acc[k] = (uint64_t)(seed + k) * 0x9e3779b97f4a7c15ull + threadIdx.x;
  for (uint32_t it = 0; it < iters; it++) {
#pragma unroll
    for (uint32_t r = 0; r < MAD_UNROLL; r++)
#pragma unroll
      for (int k = 0; k < 8; k++) acc[k] += (uint64_t)(uint32_t)acc[k] * b;
  }
  uint64_t x = 0;
#pragma unroll
  for (int k = 0; k < 8; k++) x ^= acc[k];
  if ((uint32_t)x == seed) sink[0] = (uint32_t)(x >> 32);  // keeps every chain live
}

}  // namespace

uint64_t prof_mad_count(uint32_t blocks, uint32_t iters) {
  return (uint64_t)blocks * 256 * iters * MAD_UNROLL * 8;
}

hipError_t prof_mad_rate_launch(uint32_t blocks, uint32_t iters, uint32_t* sink, hipStream_t s) {
  hipLaunchKernelGGL(mad_rate_kernel, dim3(blocks), dim3(256), 0, s, iters, 0x2545f491u, sink);
  return hipGetLastError();
}

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
