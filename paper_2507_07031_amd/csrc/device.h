// Device facts the launch planners size their grids by.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace zk {

// Compute units of the current device, queried once per device (256 when the
// query fails, the MI355X count).
inline uint32_t device_compute_units() {
  static uint32_t cus[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
    (void)hipGetLastError();
    return 256;
  }
  if (!cus[dev]) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) {
      (void)hipGetLastError();
      n = 256;
    }
    cus[dev] = (uint32_t)n;
  }
  return cus[dev];
}

// Launch schedule of the MSM and transform planners on one device (the
// autotuner's knobs; no result depends on them).  Set while no call on the
// device is being enqueued.
struct Schedule {
  uint32_t acc_max_slice = 256;      // most sorted entries per accumulating thread and round
  uint32_t acc_blocks_per_cu = 2;    // accumulation workgroups per compute unit and round
  uint32_t reduce_chunk = 0;         // buckets per running-sum chunk (0: 4, 8 or 16 by bucket count)
  uint32_t sort_chunk = 1024;        // scalars per coarse-sort workgroup
  uint32_t sort_bin_entries = 32768; // entries per coarse bin the two-level sort aims at
  uint32_t ntt_tile_log = 11;        // preferred transform tile (11: 2^11 where both passes fit it, else 2^12)
  uint32_t ntt_unit_log = 3;         // transform stages per LDS round trip: 3 (8 points a thread) or 2
  uint32_t ntt_overlap_tile_log = 11;  // tile of a transform the library runs beside other kernels
};

inline Schedule* schedule_slots() {
  static Schedule slots[64];
  return slots;
}

inline int schedule_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
    (void)hipGetLastError();
    return -1;
  }
  return dev;
}

// The current device's schedule (the defaults when there is no device).
inline Schedule device_schedule() {
  const int dev = schedule_device();
  return dev < 0 ? Schedule() : schedule_slots()[dev];
}

}  // namespace zk
