// Internal interface of the quotient kernels (quotient.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "field.h"

namespace zk {

constexpr uint32_t QUOT_MAX_LOG_BLOWUP = 4;

// On the coset s H_(B n), B = 2^log_b: the vanishing polynomial X^n - 1 takes
// the B values s^n omega_B^k - 1 (k = j mod B at point j).  zinv_r2[k] is
// the inverse of value k times 2^522 mod r (so that a Montgomery product
// with a value divided by 2^261 yields the plain quotient).
struct QuotZinv {
  f29 zinv_r2[1u << QUOT_MAX_LOG_BLOWUP];
};

// e[j] = (e[j] * f[j] - g[j]) / Z(point j), j < big, for plain canonical
// evaluations (in place into e).
hipError_t quot_mul_pointwise(uint32_t* e, const uint32_t* f, const uint32_t* g, uint64_t big, uint32_t log_b,
                              const QuotZinv& z, hipStream_t s);

// out[i] = u[i] * w^i for i < n, w^e read from split power tables
// (lo[e mod 2^14] * hi[e / 2^14], Montgomery form).
hipError_t quot_scale_powers(const uint32_t* u, uint64_t n, const f29* lo, const f29* hi, uint32_t* out,
                             hipStream_t s);

}  // namespace zk
