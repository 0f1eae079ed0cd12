// Internal interface of the KZG opening kernels (open.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace zk {

// Scratch bytes open_quotient needs for m polynomials of n coefficients.
size_t open_scratch_bytes(uint32_t m, uint64_t n);

// For m polynomials of n coefficients (polys[i*n + j], canonical words) and
// canonical x, gamma (host words):
//   ys[i] = f_i(x)                                      (m elements)
//   q     = (g - g(x)) / (X - x),  g = sum_i gamma^i f_i (n - 1 elements)
// all canonical.  gamma is ignored when m == 1.  scratch: open_scratch_bytes.
hipError_t open_quotient(const uint32_t* polys, uint32_t m, uint64_t n, const uint32_t x[8],
                         const uint32_t gamma[8], uint32_t* ys, uint32_t* q, void* scratch, hipStream_t s);

}  // namespace zk
