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

}  // namespace zk
