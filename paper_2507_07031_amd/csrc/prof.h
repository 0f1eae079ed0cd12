// Optional kernel timing: named regions bracketed by HIP events on the
// stream the kernels are launched on (enabled by zk_profile_enable).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace zk {

struct ProfToken {
  int id = -1;
};

bool prof_enabled();
void prof_set_enabled(bool on);
// Record only regions called `name` (nullptr: every region).
void prof_set_filter(const char* name);
ProfToken prof_begin(const char* name, hipStream_t s);
void prof_end(ProfToken t, hipStream_t s);
// Sum of elapsed times (ms) and count of completed regions called `name`;
// waits for their events.  reset: forget them afterwards.
int prof_read(const char* name, double* total_ms, unsigned long long* count, bool reset);

// v_mad_u64_u32 issue-rate calibration: `blocks` workgroups of 256 threads,
// prof_mad_count(blocks, iters) products in all; sink: one device word.
uint64_t prof_mad_count(uint32_t blocks, uint32_t iters);
hipError_t prof_mad_rate_launch(uint32_t blocks, uint32_t iters, uint32_t* sink, hipStream_t s);

}  // namespace zk
