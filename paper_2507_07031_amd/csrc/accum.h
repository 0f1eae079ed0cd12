// Internal interface of the accumulation-step kernels (accum.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "field.h"

namespace zk {

constexpr uint32_t ACC_MAX_D = 15;  // largest relation degree d

// G1 part of one accumulation step, every output computed by one quad:
//   C_out[i] = gamma C[i] + C2[i]                               (i < k)
//   E_out    = E2 + sum_(j=1)^(d-1) gamma^j Ej[j-1] + gamma^d E
// Points are canonical plain affine words ((0, 0) = infinity); gamma is a
// device Fr.  scratch: acc_fold_g1_scratch_bytes(k, d).
size_t acc_fold_g1_scratch_bytes(uint32_t k, uint32_t d);
hipError_t acc_fold_g1(const uint32_t* C, const uint32_t* C2, uint32_t k, const uint32_t* E, const uint32_t* E2,
                       const uint32_t* Ej, uint32_t d, const uint32_t* gamma, uint32_t* C_out, uint32_t* E_out,
                       void* scratch, hipStream_t s);

// out[j] = sum_(i<m) sigma_i P(i, j) for j < k, points P(i, j) at pts[(i k + j) * 16]
// (canonical plain affine words, (0, 0) = infinity), sigma: m canonical Fr
// words; every term on its own quad (one scalar multiple's latency), for
// m <= G1_RLC_TERMS_MAX.  scratch: g1_rlc_scratch_bytes(m, k).
constexpr uint32_t G1_RLC_TERMS_MAX = 1024;
size_t g1_rlc_scratch_bytes(uint32_t m, uint32_t k);
hipError_t g1_rlc(const uint32_t* pts, const uint32_t* sigma, uint32_t m, uint32_t k, uint32_t* out, void* scratch,
                  hipStream_t s);

// out[i] = v0[i] + sum_(t=1)^(d-1) gamma^t vmid[(t-1) len + i] + gamma^d vlast[i], i < len.
hipError_t fr_rlc(const uint32_t* v0, const uint32_t* vmid, const uint32_t* vlast, uint32_t d, uint64_t len,
                  const uint32_t* gamma, uint32_t* out, hipStream_t s);

// Challenge from a byte string: the 512-bit little-endian integer
// SHA-256(0x00 || data) || SHA-256(0x01 || data), reduced mod r.
// c_2_256: 2^256 in Montgomery form (2^256 * 2^261 mod r).
hipError_t transcript_challenge(const uint8_t* data, uint64_t bytes, const f29& c_2_256, uint32_t* out,
                                hipStream_t s);

}  // namespace zk
